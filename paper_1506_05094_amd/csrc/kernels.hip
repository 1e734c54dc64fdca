// Device kernels of libsrmd for gfx950 (MI355X).
//
// Hot path of one time step (paper sections 5-7):
//   list rebuild (only when the device flag asks for it; every kernel of the chain
//   exits at once otherwise, the paper's device-side rebuild decision of section 6):
//     k_bin      cell coordinates of every particle, cell histogram
//     k_scan     exclusive scan of the histogram -> cell start offsets
//     k_scatter  one slot per particle inside its cell (arrival order)
//     k_gather   final slot = cell start + rank of the particle id inside the cell
//                (deterministic order), gather of every per-particle array
//                (the spatial reorder of section 7)
//     k_list     Verlet list from the 5x5x5 cell stencil with cells of side
//                >= (r_c + s)/2 (section 7), copy of the sorted arrays back
//   k_step      fused pair force (t_p lanes per particle, section 3 and 5) and
//               leapfrog / Nose-Hoover update, float64 block partials of
//               potential energy, virial, kinetic energy and the largest
//               displacement; the last block to finish reduces them in a fixed
//               order, updates the thermostat and sets the rebuild flag.
#include "srmd_internal.h"

namespace srmd {

// ---------------------------------------------------------------- helpers

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Remap so that each XCD works on one contiguous range of (spatially sorted)
// particles and its L2 holds that region's positions.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

// float32 minimum image of one coordinate difference: the specified sequence
// m = rint(d * invL) (ties to even), d = fma(-m, L, d).
__device__ __forceinline__ float min_image(float d, float L, float invL) {
  const float m = __builtin_rintf(d * invL);
  return __builtin_fmaf(-m, L, d);
}

// float32 squared distance from a to b; d = b - a after the minimum image.
__device__ __forceinline__ float dist2(const float4 a, const float4 b, const SysConst &c, float &dx, float &dy,
                                       float &dz) {
  dx = min_image(b.x - a.x, c.L[0], c.invL[0]);
  dy = min_image(b.y - a.y, c.L[1], c.invL[1]);
  dz = min_image(b.z - a.z, c.L[2], c.invL[2]);
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

__device__ __forceinline__ int ptype(const float4 r) { return __float_as_int(r.w); }

__device__ __forceinline__ int cell_coord(float x, float halfL, float scale, int nc) {
  const int k = (int)floorf((x + halfL) * scale);
  return min(max(k, 0), nc - 1);
}

__device__ __forceinline__ void cell_coords(const float4 r, const SysConst &c, int &cx, int &cy, int &cz) {
  cx = cell_coord(r.x, c.halfL[0], c.cscale[0], c.nc[0]);
  cy = cell_coord(r.y, c.halfL[1], c.cscale[1], c.nc[1]);
  cz = cell_coord(r.z, c.halfL[2], c.cscale[2], c.nc[2]);
}

// Address of entry k of particle i in the tp-interleaved column-major list:
// groups of tp consecutive entries of one particle are stored contiguously, and
// consecutive particles' groups follow each other, so the tp lanes of a wave that
// serve consecutive particles read one contiguous span per iteration.  tp = 1 is
// the paper's column-major layout (section 5).
__device__ __forceinline__ long long nbl_addr(int i, int k, int tp, int nvp) {
  return (long long)(k / tp) * ((long long)nvp * tp) + (long long)i * tp + (k % tp);
}

// Pair table staged in LDS.
struct SharedPairs {
  float rc2[kMaxPairs], sig2[kMaxPairs], eps4[kMaxPairs], eps24[kMaxPairs], ushift[kMaxPairs], fc[kMaxPairs],
      rc[kMaxPairs];
};

__device__ __forceinline__ void stage_pairs(SharedPairs &sp, const SysConst &c) {
  const int t = threadIdx.x;
  if (t < kMaxPairs) {
    sp.rc2[t] = c.pt.rc2[t];
    sp.sig2[t] = c.pt.sig2[t];
    sp.eps4[t] = c.pt.eps4[t];
    sp.eps24[t] = c.pt.eps24[t];
    sp.ushift[t] = c.pt.ushift[t];
    sp.fc[t] = c.pt.fc[t];
    sp.rc[t] = c.pt.rc[t];
  }
}

// One pair contribution (12-6 Lennard-Jones, paper section 2 cutoff methods).
// Accumulates the force on i (-fr * d, with fr = F(r)/r and d = r_j - r_i), the
// pair energy u and fr * r^2 (= r . F) for the virial.
template <int METHOD>
__device__ __forceinline__ void pair_acc(const float4 pi, const float4 pj, int ti, int ntypes, const SharedPairs &sp,
                                         const SysConst &c, float &fx, float &fy, float &fz, float &u, float &w) {
  float dx, dy, dz;
  const float r2 = dist2(pi, pj, c, dx, dy, dz);
  const int ab = ti * ntypes + ptype(pj);
  if (r2 < sp.rc2[ab]) {
    const float inv_r2 = __builtin_amdgcn_rcpf(r2);
    const float s2 = sp.sig2[ab] * inv_r2;
    const float s6 = s2 * s2 * s2;
    const float s12 = s6 * s6;
    float fr = sp.eps24[ab] * __builtin_fmaf(2.0f, s12, -s6) * inv_r2;
    float e = __builtin_fmaf(sp.eps4[ab], s12 - s6, -sp.ushift[ab]);
    if (METHOD == 2) {  // shifted force: F(r) - F(rc); U(r) - U(rc) + (r - rc) F(rc)
      const float inv_r = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * inv_r;
      fr = __builtin_fmaf(-sp.fc[ab], inv_r, fr);
      e = __builtin_fmaf(r - sp.rc[ab], sp.fc[ab], e);
    }
    fx = __builtin_fmaf(-fr, dx, fx);
    fy = __builtin_fmaf(-fr, dy, fy);
    fz = __builtin_fmaf(-fr, dz, fz);
    u += e;
    w = __builtin_fmaf(fr, r2, w);
  }
}

// Force on particle i from lane t of its TP lanes (entries k = t, t+TP, ...).
template <int TP, int METHOD>
__device__ __forceinline__ void force_lane(int i, int t, const float4 pi, const float4 *__restrict__ pos,
                                           const int *__restrict__ nbl, int nn, const SharedPairs &sp,
                                           const SysConst &c, float &fx, float &fy, float &fz, float &u, float &w) {
  const int ti = ptype(pi);
  const long long stride = (long long)c.nvp * TP;
  const int *row = nbl + (long long)i * TP + t;
  int k = t;
  // two entries per iteration: both indices, then both positions, are in flight together
  for (; k + TP < nn; k += 2 * TP) {
    const int j0 = __builtin_nontemporal_load(row + (long long)(k / TP) * stride);
    const int j1 = __builtin_nontemporal_load(row + (long long)(k / TP + 1) * stride);
    const float4 p0 = pos[j0];
    const float4 p1 = pos[j1];
    pair_acc<METHOD>(pi, p0, ti, c.ntypes, sp, c, fx, fy, fz, u, w);
    pair_acc<METHOD>(pi, p1, ti, c.ntypes, sp, c, fx, fy, fz, u, w);
  }
  if (k < nn) {
    const int j0 = __builtin_nontemporal_load(row + (long long)(k / TP) * stride);
    pair_acc<METHOD>(pi, pos[j0], ti, c.ntypes, sp, c, fx, fy, fz, u, w);
  }
}

template <int TP>
__device__ __forceinline__ float lane_sum(float v) {
#pragma unroll
  for (int o = TP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, TP);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide reduction of one BlockPartial (fixed order: lanes by butterfly, then
// waves in index order), result valid in thread 0.
__device__ void block_reduce(BlockPartial &v, BlockPartial *s_waves) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v.pe = wave_sum(v.pe);
  v.w = wave_sum(v.w);
  v.ke_half = wave_sum(v.ke_half);
  v.ke_int = wave_sum(v.ke_int);
  v.disp2 = wave_max(v.disp2);
  int bad = v.nonfinite;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, 64);
  v.nonfinite = bad;
  if (lane == 0) s_waves[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    BlockPartial a = s_waves[0];
    for (int k = 1; k < nw; ++k) {
      a.pe += s_waves[k].pe;
      a.w += s_waves[k].w;
      a.ke_half += s_waves[k].ke_half;
      a.ke_int += s_waves[k].ke_int;
      a.disp2 = fmax(a.disp2, s_waves[k].disp2);
      a.nonfinite |= s_waves[k].nonfinite;
    }
    v = a;
  }
}

// Reduction of the per-block partials by one wave in a fixed order (independent of
// which block runs it).
__device__ BlockPartial reduce_partials(const BlockPartial *part, int G) {
  const int lane = threadIdx.x & 63;
  BlockPartial a{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0.0};
  for (int b = lane; b < G; b += 64) {
    const BlockPartial q = part[b];
    a.pe += q.pe;
    a.w += q.w;
    a.ke_half += q.ke_half;
    a.ke_int += q.ke_int;
    a.disp2 = fmax(a.disp2, q.disp2);
    a.nonfinite |= q.nonfinite;
  }
  a.pe = wave_sum(a.pe);
  a.w = wave_sum(a.w);
  a.ke_half = wave_sum(a.ke_half);
  a.ke_int = wave_sum(a.ke_int);
  a.disp2 = wave_max(a.disp2);
  int bad = a.nonfinite;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, 64);
  a.nonfinite = bad;
  return a;
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

// ---------------------------------------------------------------- rebuild chain

__global__ __launch_bounds__(1024) void k_bin(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= c.n) return;
  const float4 r = p.pos[cur][s];
  int cx, cy, cz;
  cell_coords(r, c, cx, cy, cz);
  const unsigned cell = (unsigned)((cz * c.nc[1] + cy) * c.nc[0] + cx);
  p.cell_of[s] = cell;
  p.slot_in_cell[s] = atomicAdd(&p.cell_count[cell], 1u);
}

// Exclusive scan of the cell histogram by one block, in tiles of blockDim.x
// cells; clears the histogram for the next build.
__global__ __launch_bounds__(1024) void k_scan(SysConst c, SysPtrs p) {
  if (p.ctl->rebuild == 0) return;
  __shared__ unsigned s_w[16];
  __shared__ unsigned s_carry;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  if (t == 0) {
    s_carry = 0;
    p.ctl->max_nbrs = 0;
    p.ctl->n_rebuilds += 1;
    p.ctl->rebuilt_this_step = 1;
  }
  __syncthreads();
  for (int base = 0; base < c.ncell; base += blockDim.x) {
    const int idx = base + t;
    const unsigned v = idx < c.ncell ? p.cell_count[idx] : 0u;
    // inclusive scan inside the wave
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    unsigned wbase = 0;
    for (int k = 0; k < wv; ++k) wbase += s_w[k];
    const unsigned excl = s_carry + wbase + x - v;
    if (idx < c.ncell) {
      p.cell_start[idx] = excl;
      p.cell_count[idx] = 0u;
    }
    __syncthreads();
    if (t == 0) {
      unsigned tot = 0;
      for (int k = 0; k < nw; ++k) tot += s_w[k];
      s_carry += tot;
    }
    __syncthreads();
  }
  if (t == 0) p.cell_start[c.ncell] = s_carry;
}

__global__ __launch_bounds__(1024) void k_scatter(SysConst c, SysPtrs p) {
  if (p.ctl->rebuild == 0) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= c.n) return;
  p.perm_tmp[p.cell_start[p.cell_of[s]] + p.slot_in_cell[s]] = (unsigned)s;
}

__global__ __launch_bounds__(1024) void k_gather(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= c.n) return;
  const unsigned cell = p.cell_of[s];
  const unsigned beg = p.cell_start[cell], end = p.cell_start[cell + 1];
  const int4 im = p.img[s];
  unsigned rank = 0;
  for (unsigned u = beg; u < end; ++u) rank += (p.img[p.perm_tmp[u]].w < im.w) ? 1u : 0u;
  const unsigned dst = beg + rank;
  p.t_pos[dst] = p.pos[cur][s];
  p.t_vel[dst] = p.vel[s];
  p.t_img[dst] = im;
  if (p.pos64) {
    p.t_pos64[3 * dst] = p.pos64[3 * s];
    p.t_pos64[3 * dst + 1] = p.pos64[3 * s + 1];
    p.t_pos64[3 * dst + 2] = p.pos64[3 * s + 2];
  }
  if (p.kahan) p.t_kahan[dst] = p.kahan[s];
}

// Verlet list of particle t (sorted slot) from the cell stencil; also moves the
// sorted arrays into place and records the build positions.
__global__ __launch_bounds__(1024) void k_list(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  if (threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  __syncthreads();
  const int t = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= c.n) return;
  const float4 r = p.t_pos[t];
  p.pos[cur][t] = r;
  p.vel[t] = p.t_vel[t];
  p.img[t] = p.t_img[t];
  p.last[t] = r;
  if (p.pos64) {
    p.pos64[3 * t] = p.t_pos64[3 * t];
    p.pos64[3 * t + 1] = p.t_pos64[3 * t + 1];
    p.pos64[3 * t + 2] = p.t_pos64[3 * t + 2];
  }
  if (p.kahan) p.kahan[t] = p.t_kahan[t];
  const int ti = ptype(r);
  int cx, cy, cz;
  cell_coords(r, c, cx, cy, cz);
  const int cc[3] = {cx, cy, cz};
  int lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (c.full_axis & (1 << k)) {
      lo[k] = 0;
      hi[k] = c.nc[k] - 1;
    } else {
      lo[k] = cc[k] - 2;
      hi[k] = cc[k] + 2;
    }
  }
  int cnt = 0;
  const int nmax = c.n_max;
  for (int oz = lo[2]; oz <= hi[2]; ++oz) {
    const int zz = (oz + c.nc[2]) % c.nc[2];
    for (int oy = lo[1]; oy <= hi[1]; ++oy) {
      const int yy = (oy + c.nc[1]) % c.nc[1];
      const int rowbase = (zz * c.nc[1] + yy) * c.nc[0];
      for (int ox = lo[0]; ox <= hi[0]; ++ox) {
        const int xx = (ox + c.nc[0]) % c.nc[0];
        const int cell = rowbase + xx;
        const unsigned beg = p.cell_start[cell], end = p.cell_start[cell + 1];
        for (unsigned u = beg; u < end; ++u) {
          if ((int)u == t) continue;
          const float4 q = p.t_pos[u];
          float dx, dy, dz;
          const float r2 = dist2(r, q, c, dx, dy, dz);
          if (r2 < s_cs2[ti * c.ntypes + ptype(q)]) {
            if (cnt < nmax) p.nbl[nbl_addr(t, cnt, c.tp, c.nvp)] = (int)u;
            ++cnt;
          }
        }
      }
    }
  }
  p.nnb[t] = min(cnt, nmax);
  if (cnt > nmax) atomicOr(&p.ctl->error, 2);
  atomicMax(&p.ctl->max_nbrs, cnt);
}

// ---------------------------------------------------------------- force only

template <int TP, int METHOD>
__global__ __launch_bounds__(1024) void k_force(SysConst c, SysPtrs p, int cur) {
  __shared__ SharedPairs sp;
  __shared__ BlockPartial s_waves[16];
  __shared__ int s_last;
  stage_pairs(sp, c);
  __syncthreads();
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int gt = lb * blockDim.x + threadIdx.x;
  const int i = gt / TP, t = gt % TP;
  const bool active = i < c.n;
  const float4 *pos = p.pos[cur];
  float fx = 0.f, fy = 0.f, fz = 0.f, u = 0.f, w = 0.f;
  if (active) {
    const float4 pi = pos[i];
    force_lane<TP, METHOD>(i, t, pi, pos, p.nbl, p.nnb[i], sp, c, fx, fy, fz, u, w);
  }
  fx = lane_sum<TP>(fx);
  fy = lane_sum<TP>(fy);
  fz = lane_sum<TP>(fz);
  u = lane_sum<TP>(u);
  w = lane_sum<TP>(w);
  BlockPartial v{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0.0};
  if (active && t == 0) {
    p.force[i] = make_float4(fx, fy, fz, 0.5f * u);
    v.pe = 0.5 * (double)u;
    v.w = (double)w / 6.0;
    const float4 vo = p.vel[i];
    const double dvx = vo.x, dvy = vo.y, dvz = vo.z;
    v.ke_half = 0.5 * c.mass[ptype(pos[i])] * (dvx * dvx + dvy * dvy + dvz * dvz);
    v.nonfinite = finite3(fx, fy, fz) ? 0 : 1;
  }
  block_reduce(v, s_waves);
  if (threadIdx.x == 0) {
    p.part[lb] = v;
    __threadfence();
    const unsigned prev = atomicAdd(&p.ctl->counter, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (threadIdx.x < 64) {
    const BlockPartial a = reduce_partials(p.part, gridDim.x);
    if (threadIdx.x == 0) {
      Thermo *th = p.thermo;
      th->pe = a.pe;
      th->virial = a.w;
      th->ke = a.ke_half;  // kinetic energy of the stored (half-step) velocities
      th->ke_half = a.ke_half;
      th->temperature = 2.0 * a.ke_half / c.g;
      th->pressure = (2.0 * a.ke_half / 3.0 + a.w) / c.volume;
      th->xi = c.thermostat ? p.ctl->xi : 0.0;
      th->xi_integral = p.ctl->xi_int;
      th->h_conserved = a.ke_half + a.pe;
      th->max_nbrs = p.ctl->max_nbrs;
      th->n_rebuilds = p.ctl->n_rebuilds;
      th->step = p.ctl->step;
      if (a.nonfinite) atomicOr(&p.ctl->error, 1);
      p.ctl->counter = 0u;
      p.ctl->rebuild = 0;
      p.ctl->rebuilt_this_step = 0;
    }
  }
}

// ---------------------------------------------------------------- fused step

template <int TP, int METHOD, int PREC>
__global__ __launch_bounds__(1024) void k_step(SysConst c, SysPtrs p, int cur) {
  __shared__ SharedPairs sp;
  __shared__ BlockPartial s_waves[16];
  __shared__ int s_last;
  stage_pairs(sp, c);
  __syncthreads();
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int gt = lb * blockDim.x + threadIdx.x;
  const int i = gt / TP, t = gt % TP;
  const bool active = i < c.n;
  const float4 *pos = p.pos[cur];
  float fx = 0.f, fy = 0.f, fz = 0.f, u = 0.f, w = 0.f;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  if (active) {
    pi = pos[i];
    force_lane<TP, METHOD>(i, t, pi, pos, p.nbl, p.nnb[i], sp, c, fx, fy, fz, u, w);
  }
  fx = lane_sum<TP>(fx);
  fy = lane_sum<TP>(fy);
  fz = lane_sum<TP>(fz);
  u = lane_sum<TP>(u);
  w = lane_sum<TP>(w);
  const double xi = p.ctl->xi;
  BlockPartial v{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0.0};
  if (active && t == 0) {
    const int ti = ptype(pi);
    // v(n+1/2) = [v(n-1/2) (1 - xi dt/2) + F/m dt] / (1 + xi dt/2); a = b = 1 without thermostat
    const double hx = c.thermostat ? 0.5 * xi * c.dtd : 0.0;
    const float a = (float)(1.0 - hx);
    const float ib = (float)(1.0 / (1.0 + hx));
    const float dtm = c.dt * c.inv_mass[ti];
    const float4 vo = p.vel[i];
    const float vx = __builtin_fmaf(vo.x, a, fx * dtm) * ib;
    const float vy = __builtin_fmaf(vo.y, a, fy * dtm) * ib;
    const float vz = __builtin_fmaf(vo.z, a, fz * dtm) * ib;
    p.vel[i] = make_float4(vx, vy, vz, vo.w);
    p.force[i] = make_float4(fx, fy, fz, 0.5f * u);
    int4 im = p.img[i];
    float4 rn;
    rn.w = pi.w;
    if (PREC == 2) {  // float64 master positions
      double x = p.pos64[3 * i] + (double)vx * c.dtd;
      double y = p.pos64[3 * i + 1] + (double)vy * c.dtd;
      double z = p.pos64[3 * i + 2] + (double)vz * c.dtd;
      if (x >= 0.5 * c.Ld[0]) { x -= c.Ld[0]; im.x += 1; } else if (x < -0.5 * c.Ld[0]) { x += c.Ld[0]; im.x -= 1; }
      if (y >= 0.5 * c.Ld[1]) { y -= c.Ld[1]; im.y += 1; } else if (y < -0.5 * c.Ld[1]) { y += c.Ld[1]; im.y -= 1; }
      if (z >= 0.5 * c.Ld[2]) { z -= c.Ld[2]; im.z += 1; } else if (z < -0.5 * c.Ld[2]) { z += c.Ld[2]; im.z -= 1; }
      p.pos64[3 * i] = x;
      p.pos64[3 * i + 1] = y;
      p.pos64[3 * i + 2] = z;
      rn.x = (float)x;
      rn.y = (float)y;
      rn.z = (float)z;
      // the float32 copy may round up onto +L/2; use the periodic twin -L/2
      if (rn.x >= c.halfL[0]) rn.x = -c.halfL[0];
      if (rn.y >= c.halfL[1]) rn.y = -c.halfL[1];
      if (rn.z >= c.halfL[2]) rn.z = -c.halfL[2];
    } else {
      float x, y, z;
      if (PREC == 1) {  // compensated update: y = v dt - c; t = r + y; c = (t - r) - y
        float4 kc = p.kahan[i];
        const float yx = vx * c.dt - kc.x, yy = vy * c.dt - kc.y, yz = vz * c.dt - kc.z;
        x = pi.x + yx;
        y = pi.y + yy;
        z = pi.z + yz;
        kc.x = (x - pi.x) - yx;
        kc.y = (y - pi.y) - yy;
        kc.z = (z - pi.z) - yz;
        p.kahan[i] = kc;
      } else {
        x = __builtin_fmaf(vx, c.dt, pi.x);
        y = __builtin_fmaf(vy, c.dt, pi.y);
        z = __builtin_fmaf(vz, c.dt, pi.z);
      }
      // wrap into [-L/2, L/2); both corrections are exact (Sterbenz)
      if (x >= c.halfL[0]) { x -= c.L[0]; im.x += 1; } else if (x < -c.halfL[0]) { x += c.L[0]; im.x -= 1; }
      if (y >= c.halfL[1]) { y -= c.L[1]; im.y += 1; } else if (y < -c.halfL[1]) { y += c.L[1]; im.y -= 1; }
      if (z >= c.halfL[2]) { z -= c.L[2]; im.z += 1; } else if (z < -c.halfL[2]) { z += c.L[2]; im.z -= 1; }
      rn.x = x;
      rn.y = y;
      rn.z = z;
    }
    p.pos[cur ^ 1][i] = rn;
    p.img[i] = im;
    // float64 reductions
    const double m = c.mass[ti];
    const double dvx = vx, dvy = vy, dvz = vz;
    v.ke_half = 0.5 * m * (dvx * dvx + dvy * dvy + dvz * dvz);
    const double mx = 0.5 * ((double)vo.x + dvx), my = 0.5 * ((double)vo.y + dvy), mz = 0.5 * ((double)vo.z + dvz);
    v.ke_int = 0.5 * m * (mx * mx + my * my + mz * mz);
    v.pe = 0.5 * (double)u;
    v.w = (double)w / 6.0;
    // displacement since the last build: float64 from the float32 positions
    const float4 l0 = p.last[i];
    double ddx = (double)rn.x - (double)l0.x, ddy = (double)rn.y - (double)l0.y, ddz = (double)rn.z - (double)l0.z;
    ddx -= c.Ld[0] * rint(ddx / c.Ld[0]);
    ddy -= c.Ld[1] * rint(ddy / c.Ld[1]);
    ddz -= c.Ld[2] * rint(ddz / c.Ld[2]);
    v.disp2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
    v.nonfinite = (finite3(fx, fy, fz) && finite3(rn.x, rn.y, rn.z)) ? 0 : 1;
  }
  block_reduce(v, s_waves);
  if (threadIdx.x == 0) {
    p.part[lb] = v;
    __threadfence();
    const unsigned prev = atomicAdd(&p.ctl->counter, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (threadIdx.x < 64) {
    const BlockPartial a = reduce_partials(p.part, gridDim.x);
    if (threadIdx.x == 0) {
      Control *ctl = p.ctl;
      Thermo rec;
      rec.pe = a.pe;
      rec.ke = a.ke_int;
      rec.virial = a.w;
      rec.temperature = 2.0 * a.ke_int / c.g;
      rec.pressure = (2.0 * a.ke_int / 3.0 + a.w) / c.volume;
      rec.xi = c.thermostat ? xi : 0.0;
      rec.xi_integral = ctl->xi_int;
      rec.h_conserved = a.ke_int + a.pe;
      if (c.thermostat && c.inv_tau2 > 0.0)
        rec.h_conserved += c.g * c.T0 * (xi * xi / (2.0 * c.inv_tau2) + ctl->xi_int);
      rec.ke_half = a.ke_half;
      rec.step = ctl->step;
      rec.n_rebuilds = ctl->n_rebuilds;
      rec.max_nbrs = ctl->max_nbrs;
      rec.reserved = 0;
      *p.thermo = rec;
      if (ctl->thermo_every > 0 && (ctl->step % ctl->thermo_every) == 0 && ctl->n_records < ctl->trace_cap) {
        p.trace[ctl->n_records] = rec;
        ctl->n_records += 1;
      }
      if (c.thermostat) {
        const double th = 2.0 * a.ke_half / c.g;
        const double xn = xi + c.dtd * (th / c.T0 - 1.0) * c.inv_tau2;
        ctl->xi_int += c.dtd * (xi + xn) * 0.5;
        ctl->xi = xn;
      }
      ctl->step += 1;
      ctl->rebuild = (a.disp2 > c.half_skin2) ? 1 : 0;
      ctl->rebuilt_this_step = 0;
      if (a.nonfinite) ctl->error |= 1;
      ctl->counter = 0u;
    }
  }
}

// ---------------------------------------------------------------- launchers

template <int TP>
static hipError_t launch_step_tp(int method, int prec, dim3 g, dim3 b, hipStream_t st, const SysConst &c,
                                 const SysPtrs &p, int cur) {
#define SRMD_STEP_CASE(M, P)                                                   \
  if (method == M && prec == P) {                                              \
    hipLaunchKernelGGL((k_step<TP, M, P>), g, b, 0, st, c, p, cur);            \
    return hipGetLastError();                                                  \
  }
  SRMD_STEP_CASE(0, 0) SRMD_STEP_CASE(0, 1) SRMD_STEP_CASE(0, 2)
  SRMD_STEP_CASE(1, 0) SRMD_STEP_CASE(1, 1) SRMD_STEP_CASE(1, 2)
  SRMD_STEP_CASE(2, 0) SRMD_STEP_CASE(2, 1) SRMD_STEP_CASE(2, 2)
#undef SRMD_STEP_CASE
  return hipErrorInvalidValue;
}

template <int TP>
static hipError_t launch_force_tp(int method, dim3 g, dim3 b, hipStream_t st, const SysConst &c, const SysPtrs &p,
                                  int cur) {
  if (method == 0) hipLaunchKernelGGL((k_force<TP, 0>), g, b, 0, st, c, p, cur);
  else if (method == 1) hipLaunchKernelGGL((k_force<TP, 1>), g, b, 0, st, c, p, cur);
  else if (method == 2) hipLaunchKernelGGL((k_force<TP, 2>), g, b, 0, st, c, p, cur);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_step(int tp, int method, int prec, int blocks, int threads, hipStream_t st, const SysConst &c,
                       const SysPtrs &p, int cur) {
  const dim3 g(blocks), b(threads);
  switch (tp) {
    case 1: return launch_step_tp<1>(method, prec, g, b, st, c, p, cur);
    case 2: return launch_step_tp<2>(method, prec, g, b, st, c, p, cur);
    case 4: return launch_step_tp<4>(method, prec, g, b, st, c, p, cur);
    case 8: return launch_step_tp<8>(method, prec, g, b, st, c, p, cur);
    case 16: return launch_step_tp<16>(method, prec, g, b, st, c, p, cur);
    case 32: return launch_step_tp<32>(method, prec, g, b, st, c, p, cur);
    case 64: return launch_step_tp<64>(method, prec, g, b, st, c, p, cur);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_force(int tp, int method, int blocks, int threads, hipStream_t st, const SysConst &c,
                        const SysPtrs &p, int cur) {
  const dim3 g(blocks), b(threads);
  switch (tp) {
    case 1: return launch_force_tp<1>(method, g, b, st, c, p, cur);
    case 2: return launch_force_tp<2>(method, g, b, st, c, p, cur);
    case 4: return launch_force_tp<4>(method, g, b, st, c, p, cur);
    case 8: return launch_force_tp<8>(method, g, b, st, c, p, cur);
    case 16: return launch_force_tp<16>(method, g, b, st, c, p, cur);
    case 32: return launch_force_tp<32>(method, g, b, st, c, p, cur);
    case 64: return launch_force_tp<64>(method, g, b, st, c, p, cur);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rebuild(hipStream_t st, const SysConst &c, const SysPtrs &p, int cur) {
  const int tb = 256;
  const int nb = (c.n + tb - 1) / tb;
  hipLaunchKernelGGL(k_bin, dim3(nb), dim3(tb), 0, st, c, p, cur);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, c, p);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(tb), 0, st, c, p);
  hipLaunchKernelGGL(k_gather, dim3(nb), dim3(tb), 0, st, c, p, cur);
  hipLaunchKernelGGL(k_list, dim3(nb), dim3(tb), 0, st, c, p, cur);
  return hipGetLastError();
}

}  // namespace srmd
