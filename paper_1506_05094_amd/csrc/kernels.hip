// Device kernels of libsrmd for gfx950 (MI355X).
//
// One time step (paper sections 5-7) runs in one of two forms with the same
// per-particle arithmetic in the same order, so both give the same trajectory bit
// for bit at the same launch shape.
//
// Launch chains, captured in HIP graphs; the decision to rebuild the neighbour list
// lives on the device (the paper's device-side flag of section 6), so no step needs
// the host:
//   list rebuild, only when the flag is set (every kernel exits at once otherwise):
//     small systems: the spatial sort already ran at the end of the previous step
//                    (k_finish), so only the list kernel runs here;
//     large systems: k_bin (cells, arrival slots, tile counts), k_scan (cell
//                    offsets, one workgroup per tile), k_scatter, k_gather
//                    (deterministic rank by particle id, gather of every
//                    per-particle array: the reorder of section 7), then the list
//                    kernel;
//     list kernels: k_list_wave (a wave per particle), k_list_cell (a wave per
//                    cell), k_list_thread (a thread per particle), k_list_allpairs
//                    (all pairs in index order, no sort: the O(N^2) builder of
//                    section 6);
//   k_step    pair forces with t_p lanes per particle (sections 3 and 5) fused with
//             the leapfrog / Nose-Hoover update; float64 partial sums per block;
//   k_finish  one workgroup: fixed-order float64 reduction of the partials,
//             thermostat update, thermodynamic record, the displacement test that
//             sets the rebuild flag (section 6), and for small systems the whole
//             spatial sort in LDS when a rebuild is due.
//
// Persistent (k_multi): every step of a call in one cooperative launch of 500
// steps, a system split over several workgroups separated by grid barriers, or many
// systems (a batch of replicas) over the workgroups; the same phases as above run
// inside it.
#include <algorithm>

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

// Cell coordinate along one axis, clamped to [0, nc - 1] in float32 before the
// conversion: x + L/2 can round to L, and a non-finite coordinate (a blown-up run,
// reported through the error word) lands in cell 0 (fmaxf returns the non-NaN
// operand), so no input can produce a cell index outside the grid.
__device__ __forceinline__ int cell_coord(float x, float halfL, float scale, int nc) {
  const float f = fminf(fmaxf(floorf((x + halfL) * scale), 0.0f), (float)(nc - 1));
  return (int)f;
}

// Native 4-vectors, for whole-element copies that stay in registers.
typedef float raw_f4 __attribute__((ext_vector_type(4)));
typedef int raw_i4 __attribute__((ext_vector_type(4)));

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

// The x extent of one stencil row: up to two runs of consecutive cells
// [a0, a1] and [b0, b1] (the second one only when the +-2 window wraps round the
// box), in the order dx = -2 .. +2; every cell when the axis has fewer than 5.
__device__ __forceinline__ void row_runs(int cx, int nx, bool full, int &a0, int &a1, int &b0, int &b1) {
  b0 = 0;
  b1 = -1;
  if (full) {
    a0 = 0;
    a1 = nx - 1;
    return;
  }
  const int lo = cx - 2, hi = cx + 2;
  if (lo < 0) {
    a0 = lo + nx;
    a1 = nx - 1;
    b0 = 0;
    b1 = hi;
  } else if (hi >= nx) {
    a0 = lo;
    a1 = nx - 1;
    b0 = 0;
    b1 = hi - nx;
  } else {
    a0 = lo;
    a1 = hi;
  }
}

// Pair table staged in LDS, one 32-byte row per type pair so that a pair's
// constants arrive in two 16-byte LDS reads.
struct alignas(16) PairRow {
  float rc2, sig2, eps24, eps4;  // rc^2, sigma^2, 24 eps, 4 eps
  float ushift, fc, rc, pad;     // U(rc), F(rc), rc
};

// Constants of the shifted-force Coulomb term of a type pair (kernel method 3).
struct alignas(16) CoulRow {
  float qq, rcc2, inv_rcc2, two_inv_rcc;  // q_a q_b, r_cc^2, 1 / r_cc^2, 2 / r_cc
};

// Constants of the two-power potential of a type pair (kernel method 4): B, n B,
// and the half exponents m/2, n/2 (A and m A are in the PairRow's eps4 and eps24).
struct alignas(16) MieRow {
  float b, nb;
  int hm, hn;
};

// Constants of a further potential of a type pair (kernel method 5).
struct alignas(16) GenRow {
  float g0, g1, g2, g3;
};

struct SharedPairs {
  PairRow row[kMaxPairs];
  CoulRow crow[kMaxPairs];
  MieRow mrow[kMaxPairs];
  GenRow grow[kMaxPairs];
};

__device__ __forceinline__ void stage_pairs(SharedPairs &sp, const SysConst &c) {
  const int t = threadIdx.x;
  if (t < kMaxPairs) {
    PairRow r;
    r.rc2 = c.pt.rc2[t];
    r.sig2 = c.pt.sig2[t];
    r.eps24 = c.pt.eps24[t];
    r.eps4 = c.pt.eps4[t];
    r.ushift = c.pt.ushift[t];
    r.fc = c.pt.fc[t];
    r.rc = c.pt.rc[t];
    r.pad = 0.f;
    sp.row[t] = r;
    CoulRow q;
    q.qq = c.pt.qq[t];
    q.rcc2 = c.pt.rcc2;
    q.inv_rcc2 = c.pt.inv_rcc2;
    q.two_inv_rcc = c.pt.two_inv_rcc;
    sp.crow[t] = q;
    MieRow g;
    g.b = c.pt.mie_b[t];
    g.nb = c.pt.mie_nb[t];
    g.hm = c.pt.mie_hm[t];
    g.hn = c.pt.mie_hn[t];
    sp.mrow[t] = g;
    sp.grow[t] = GenRow{c.pt.gen[t][0], c.pt.gen[t][1], c.pt.gen[t][2], c.pt.gen[t][3]};
  }
}

// Position of particle i widened once for the float64 coordinate differences.
struct Wide {
  double x, y, z;
};

__device__ __forceinline__ Wide widen(const float4 p) { return Wide{(double)p.x, (double)p.y, (double)p.z}; }

// One pair contribution (12-6 Lennard-Jones, paper section 2 cutoff methods).
// The in/out decision uses the specified float32 squared distance (the same bits
// as the list build and the CPU reference).  The value uses the coordinate
// differences recomputed in float64 with the same image shift and rounded once to
// float32: across the periodic boundary x_j - x_i is close to L, and rounding it
// in float32 first would cost about ulp(L/2) of absolute accuracy.
// Accumulates the force on i (-fr * d, with fr = F(r)/r and d = r_j - r_i), the
// pair energy u and fr * r^2 (= r . F) for the virial.
// x^h for 0 <= h < 32 by binary exponentiation (five squarings, fixed order).
__device__ __forceinline__ float pow_int(float x, int h) {
  float r = 1.0f;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (h & (1 << k)) r *= x;
    x *= x;
  }
  return r;
}

// Energy u and force over distance fr = F(r)/r (F = -dU/dr, positive repulsive) of
// the further pair potentials of paper section 2 (the paper names them only; these
// are the textbook forms), in float32 from the pair's constants g (kind uniform over
// the system):
//  2 Yukawa        U = eps (sig/r) exp(-kappa (r - sig)) = g0 exp(-g1 r) / r
//                  (g0 = eps sig exp(kappa sig), g1 = kappa)
//  3 Buckingham    U = A exp(-r/rho) - C / r^6               (g0 = A, g1 = 1/rho, g2 = C)
//  4 Gaussian core U = eps exp(-(r/sig)^2)                    (g0 = eps, g1 = 1/sig^2)
//  5 Dzugutov      U = eps [5.82 (x^-16 - 1.28) exp(1.1 / (x - 1.87)) (x < 1.87)
//                         + 1.28 exp(0.27 / (x - 1.94)) (x < 1.94)],  x = r/sig
//                                                            (g0 = eps, g1 = 1/sig)
//  6 Girifalco     U = -alpha [1/(s(s-1)^3) + 1/(s(s+1)^3) - 2/s^4]
//                      + beta [1/(s(s-1)^9) + 1/(s(s+1)^9) - 2/s^10],  s = r/d
//                                                            (g0 = alpha, g1 = beta, g2 = 1/d)
__device__ __forceinline__ void pair_further(int kind, const GenRow &g, float r, float inv_r, float &u, float &fr) {
  const float inv_r2 = inv_r * inv_r;
  if (kind == 2) {
    u = g.g0 * expf(-g.g1 * r) * inv_r;
    fr = u * __builtin_fmaf(g.g1, r, 1.0f) * inv_r2;
  } else if (kind == 3) {
    const float e = g.g0 * expf(-g.g1 * r);
    const float d6 = g.g2 * inv_r2 * inv_r2 * inv_r2;
    u = e - d6;
    fr = (e * g.g1 * inv_r - 6.0f * d6 * inv_r2);
  } else if (kind == 4) {
    const float e = g.g0 * expf(-r * r * g.g1);
    u = e;
    fr = 2.0f * g.g1 * e;
  } else if (kind == 5) {
    const float x = r * g.g1;
    float uu = 0.0f, du = 0.0f;
    if (x < 1.87f) {
      const float q = 1.0f / (x - 1.87f);
      const float e = expf(1.1f * q);
      const float ix2 = 1.0f / (x * x);
      const float xm = pow_int(ix2, 8);
      uu = 5.82f * (xm - 1.28f) * e;
      du = 5.82f * e * (-16.0f * xm / x - (xm - 1.28f) * 1.1f * q * q);
    }
    if (x < 1.94f) {
      const float q = 1.0f / (x - 1.94f);
      const float e = 1.28f * expf(0.27f * q);
      uu += e;
      du -= e * 0.27f * q * q;
    }
    u = g.g0 * uu;
    fr = -g.g0 * du * g.g1 * inv_r;
  } else {
    const float s = r * g.g2, is = 1.0f / s;
    const float ia = 1.0f / (s - 1.0f), ib = 1.0f / (s + 1.0f);
    const float ia3 = ia * ia * ia, ib3 = ib * ib * ib, ia9 = ia3 * ia3 * ia3, ib9 = ib3 * ib3 * ib3;
    const float is4 = is * is * is * is, is10 = is4 * is4 * is * is;
    const float att = is * (ia3 + ib3) - 2.0f * is4;
    const float rep = is * (ia9 + ib9) - 2.0f * is10;
    const float datt = -is * is * (ia3 + ib3) - 3.0f * is * (ia3 * ia + ib3 * ib) + 8.0f * is4 * is;
    const float drep = -is * is * (ia9 + ib9) - 9.0f * is * (ia9 * ia + ib9 * ib) + 20.0f * is10 * is;
    u = -g.g0 * att + g.g1 * rep;
    fr = (g.g0 * datt - g.g1 * drep) * g.g2 * inv_r;
  }
}

template <int METHOD>
__device__ __forceinline__ void pair_acc(const float4 pi, const Wide &wi, const float4 pj, int ti, int ntypes,
                                         const SharedPairs &sp, const SysConst &c, float &fx, float &fy, float &fz,
                                         float &u, float &w) {
  const float ex = pj.x - pi.x, ey = pj.y - pi.y, ez = pj.z - pi.z;
  const float mx = __builtin_rintf(ex * c.invL[0]), my = __builtin_rintf(ey * c.invL[1]),
              mz = __builtin_rintf(ez * c.invL[2]);
  float dx = __builtin_fmaf(-mx, c.L[0], ex), dy = __builtin_fmaf(-my, c.L[1], ey), dz = __builtin_fmaf(-mz, c.L[2], ez);
  const float r2s = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  const int pidx = ti * ntypes + ptype(pj);
  const PairRow &pr = sp.row[pidx];
  if (METHOD == 4) {
    // two-power potential A s^m - B s^n, s = sigma/r, with the cutoff method carried
    // by U(rc) (zero when truncated) and F(rc) (nonzero for shifted force only)
    if (r2s < pr.rc2) {
      dx = (float)(((double)pj.x - wi.x) - (double)mx * c.Ld[0]);
      dy = (float)(((double)pj.y - wi.y) - (double)my * c.Ld[1]);
      dz = (float)(((double)pj.z - wi.z) - (double)mz * c.Ld[2]);
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      const float inv_r2 = __builtin_amdgcn_rcpf(r2);
      const MieRow &mr = sp.mrow[pidx];
      const float s2 = pr.sig2 * inv_r2;
      const float sm = pow_int(s2, mr.hm), sn = pow_int(s2, mr.hn);
      float fr = (pr.eps24 * sm - mr.nb * sn) * inv_r2;
      float e = pr.eps4 * sm - mr.b * sn - pr.ushift;
      const float inv_r = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * inv_r;
      fr = __builtin_fmaf(-pr.fc, inv_r, fr);
      e = __builtin_fmaf(r - pr.rc, pr.fc, e);
      fx = __builtin_fmaf(-fr, dx, fx);
      fy = __builtin_fmaf(-fr, dy, fy);
      fz = __builtin_fmaf(-fr, dz, fz);
      u += e;
      w = __builtin_fmaf(fr, r2, w);
    }
    return;
  }
  if (METHOD == 5) {
    // a further potential of paper section 2, cutoff method by U(rc) and F(rc)
    if (r2s < pr.rc2) {
      dx = (float)(((double)pj.x - wi.x) - (double)mx * c.Ld[0]);
      dy = (float)(((double)pj.y - wi.y) - (double)my * c.Ld[1]);
      dz = (float)(((double)pj.z - wi.z) - (double)mz * c.Ld[2]);
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      const float inv_r = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * inv_r;
      float e, fr;
      pair_further(c.pot_kind, sp.grow[pidx], r, inv_r, e, fr);
      fr = __builtin_fmaf(-pr.fc, inv_r, fr);
      e = __builtin_fmaf(r - pr.rc, pr.fc, e - pr.ushift);
      fx = __builtin_fmaf(-fr, dx, fx);
      fy = __builtin_fmaf(-fr, dy, fy);
      fz = __builtin_fmaf(-fr, dz, fz);
      u += e;
      w = __builtin_fmaf(fr, r2, w);
    }
    return;
  }
  if (METHOD == 3) {
    // shifted-force Lennard-Jones inside r_c,ab plus shifted-force Coulomb inside r_cc
    // (paper section 9): q_a q_b (1/r - 1/r_cc + (r - r_cc)/r_cc^2), force
    // q_a q_b (1/r^2 - 1/r_cc^2); each term has its own float32 in/out decision
    const CoulRow &cr = sp.crow[pidx];
    const bool in_lj = r2s < pr.rc2, in_c = r2s < cr.rcc2;
    if (in_lj || in_c) {
      dx = (float)(((double)pj.x - wi.x) - (double)mx * c.Ld[0]);
      dy = (float)(((double)pj.y - wi.y) - (double)my * c.Ld[1]);
      dz = (float)(((double)pj.z - wi.z) - (double)mz * c.Ld[2]);
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      const float inv_r2 = __builtin_amdgcn_rcpf(r2);
      const float inv_r = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * inv_r;
      float fr = 0.f, e = 0.f;
      if (in_lj) {
        const float s2 = pr.sig2 * inv_r2;
        const float s6 = s2 * s2 * s2;
        const float s12 = s6 * s6;
        fr = __builtin_fmaf(-pr.fc, inv_r, pr.eps24 * __builtin_fmaf(2.0f, s12, -s6) * inv_r2);
        e = __builtin_fmaf(r - pr.rc, pr.fc, __builtin_fmaf(pr.eps4, s12 - s6, -pr.ushift));
      }
      if (in_c) {
        fr = __builtin_fmaf(cr.qq * inv_r, inv_r2 - cr.inv_rcc2, fr);
        e = __builtin_fmaf(cr.qq, __builtin_fmaf(r, cr.inv_rcc2, inv_r) - cr.two_inv_rcc, e);
      }
      fx = __builtin_fmaf(-fr, dx, fx);
      fy = __builtin_fmaf(-fr, dy, fy);
      fz = __builtin_fmaf(-fr, dz, fz);
      u += e;
      w = __builtin_fmaf(fr, r2, w);
    }
    return;
  }
  if (r2s < pr.rc2) {
    dx = (float)(((double)pj.x - wi.x) - (double)mx * c.Ld[0]);
    dy = (float)(((double)pj.y - wi.y) - (double)my * c.Ld[1]);
    dz = (float)(((double)pj.z - wi.z) - (double)mz * c.Ld[2]);
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float inv_r2 = __builtin_amdgcn_rcpf(r2);
    const float s2 = pr.sig2 * inv_r2;
    const float s6 = s2 * s2 * s2;
    const float s12 = s6 * s6;
    float fr = pr.eps24 * __builtin_fmaf(2.0f, s12, -s6) * inv_r2;
    float e = __builtin_fmaf(pr.eps4, s12 - s6, -pr.ushift);
    if (METHOD == 2) {  // shifted force: F(r) - F(rc); U(r) - U(rc) + (r - rc) F(rc)
      const float inv_r = __builtin_amdgcn_rsqf(r2);
      const float r = r2 * inv_r;
      fr = __builtin_fmaf(-pr.fc, inv_r, fr);
      e = __builtin_fmaf(r - pr.rc, pr.fc, e);
    }
    fx = __builtin_fmaf(-fr, dx, fx);
    fy = __builtin_fmaf(-fr, dy, fy);
    fz = __builtin_fmaf(-fr, dz, fz);
    u += e;
    w = __builtin_fmaf(fr, r2, w);
  }
}

// Force on particle i from lane t of its TP lanes (entries k = t, t+TP, ...).
// The lane's entries are taken B at a time: B list indices are loaded together,
// then the B neighbour positions, so a batch costs two memory round trips instead
// of two per entry (the paper prefetches one entry ahead, section 5; on MI355X the
// latency of a dependent load chain dominates, so many loads go in flight).  The
// first batch is issued before the list length arrives (clamped to the capacity
// n_max / TP of a lane), so the length and the first indices share a round trip.
template <int TP, int METHOD, int B, bool PF = false, class IdxPtr>
__device__ __forceinline__ void force_lane(int i, int t, const float4 pi, const float4 *__restrict__ pos,
                                           IdxPtr nbl, IdxPtr nnb, const SharedPairs &sp, const SysConst &c,
                                           float &fx, float &fy, float &fz, float &u, float &w) {
  const int ti = ptype(pi);
  const Wide wi = widen(pi);
  const long long stride = (long long)c.nvp * TP;
  const IdxPtr row = nbl + (long long)i * TP + t;
  const int cap = c.n_max / TP;  // entries of one lane the list can hold
  int j[B];
#pragma unroll
  for (int b = 0; b < B; ++b) j[b] = __builtin_nontemporal_load(row + (long long)min(b, cap - 1) * stride);
  const int nn = nnb[i];
  const int mine = nn > t ? (nn - t + TP - 1) / TP : 0;  // entries of this lane
  for (int m0 = 0; m0 < mine; m0 += B) {
    if (!PF && m0 > 0) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        // every load is issued (clamped to the lane's last entry) so none waits behind a branch
        const int mm = min(m0 + b, mine - 1);
        j[b] = __builtin_nontemporal_load(row + (long long)mm * stride);
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (m0 + b >= mine) j[b] = -1;
    float4 q[B];
#pragma unroll
    for (int b = 0; b < B; ++b) q[b] = pos[j[b] >= 0 ? j[b] : i];
    // PF: the next batch's indices are issued after this batch's positions, so they
    // arrive while this batch is evaluated (and a wait for the positions does not wait
    // for them)
    int jn[PF ? B : 1];
    if (PF && m0 + B < mine) {
#pragma unroll
      for (int b = 0; b < B; ++b) jn[b] = __builtin_nontemporal_load(row + (long long)min(m0 + B + b, mine - 1) * stride);
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (j[b] >= 0) pair_acc<METHOD>(pi, wi, q[b], ti, c.ntypes, sp, c, fx, fy, fz, u, w);
    if (PF && m0 + B < mine) {
#pragma unroll
      for (int b = 0; b < B; ++b) j[b] = jn[b];
    }
  }
}

// List entries of one lane taken together: about the entries a lane has at liquid
// densities (90 per particle / TP), so that few slots of the last batch idle.
template <int TP>
struct Batch {
  static constexpr int value = TP <= 2 ? 16 : TP == 4 ? 8 : TP == 8 ? 16 : TP == 16 ? 8 : TP == 32 ? 4 : 2;
};

// The launch-chain kernels take at most 8 entries per batch and prefetch the next
// batch's indices, so two batches' loads are in flight within 128 registers (the
// persistent kernel, at 2 waves per SIMD, keeps the full batches).
template <int TP>
struct StepBatch {
  static constexpr int value = Batch<TP>::value > 8 ? 8 : Batch<TP>::value;
};

// The value of lane (this lane) ^ O, O a power of two below 64, by VALU lane
// exchanges: quad permutations for 1 and 2, two bank-masked row shifts for 4, a
// row rotation for 8, and the row and half-wave swaps of gfx950 for 16 and 32.
template <int O>
__device__ __forceinline__ unsigned xor_lane(unsigned v) {
  if constexpr (O == 1) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
  } else if constexpr (O == 2) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
  } else if constexpr (O == 4) {
    // lanes 0-3 and 8-11 of a row read lane + 4 (row_shl:4), lanes 4-7 and 12-15 lane - 4 (row_shr:4)
    const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0x5, false);
    return (unsigned)__builtin_amdgcn_update_dpp(t, (int)v, 0x114, 0xF, 0xA, false);
  } else if constexpr (O == 8) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (O == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // odd rows <-> even rows
    return ((threadIdx.x >> 4) & 1) ? r[0] : r[1];
  } else {
    static_assert(O == 32, "xor_lane: O must be 1, 2, 4, 8, 16 or 32");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);  // upper half <-> lower half
    return ((threadIdx.x >> 5) & 1) ? r[0] : r[1];
  }
}

template <int O>
__device__ __forceinline__ float xor_lane(float v) {
  return __uint_as_float(xor_lane<O>(__float_as_uint(v)));
}

// Sum over the TP lanes of a particle: the butterfly lane ^ TP/2, ..., lane ^ 1 (the
// whole wave must be active).
template <int TP, int O = TP / 2>
__device__ __forceinline__ float lane_sum(float v) {
  if constexpr (O == 0) {
    return v;
  } else {
    return lane_sum<TP, O / 2>(v + xor_lane<O>(v));
  }
}

// Wave-wide reductions by DPP lane swizzles (VALU operand exchanges, no LDS round
// trip as in a shuffle).  Within each 16-lane row: the quad exchanges lane ^ 1 and
// lane ^ 2, the half-row mirror (lane i with 7 - i of its 8) and the row mirror
// (i with 15 - i), each pairing two disjoint halves, so that every lane of a row
// ends with the row's total, bitwise the same in all 16 (each step combines the
// same two values in either order).  Then lane 15 of rows 0 and 2 is combined into
// rows 1 and 3, and lane 31 into rows 2 and 3, so lane 63 holds
// (row 3 + row 2) + (row 1 + row 0), which is read back to every lane.  Lanes of the
// rows a broadcast does not reach combine with the identity.  The whole wave must
// be active.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppMirror = 0x140;     // row_mirror
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppBcast15 = 0x142;    // row_bcast:15
constexpr int kDppBcast31 = 0x143;    // row_bcast:31

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp32(unsigned old, unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long old, unsigned long long v) {
  const unsigned lo = dpp32<CTRL, ROWS>((unsigned)old, (unsigned)v);
  const unsigned hi = dpp32<CTRL, ROWS>((unsigned)(old >> 32), (unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

template <class Op>
__device__ __forceinline__ unsigned long long wave_reduce64(unsigned long long v, unsigned long long id, Op op) {
  v = op(v, dpp64<kDppXor1, 0xF>(id, v));
  v = op(v, dpp64<kDppXor2, 0xF>(id, v));
  v = op(v, dpp64<kDppHalfMirror, 0xF>(id, v));
  v = op(v, dpp64<kDppMirror, 0xF>(id, v));
  v = op(v, dpp64<kDppBcast15, 0xA>(id, v));
  v = op(v, dpp64<kDppBcast31, 0xC>(id, v));
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ double bits_f64(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long f64_bits(double d) { return (unsigned long long)__double_as_longlong(d); }

__device__ __forceinline__ double wave_sum(double v) {
  return bits_f64(wave_reduce64(f64_bits(v), f64_bits(0.0), [](unsigned long long a, unsigned long long b) {
    return f64_bits(bits_f64(a) + bits_f64(b));
  }));
}

__device__ __forceinline__ double wave_max(double v) {
  return bits_f64(wave_reduce64(f64_bits(v), f64_bits(-__builtin_inf()), [](unsigned long long a, unsigned long long b) {
    return f64_bits(fmax(bits_f64(a), bits_f64(b)));
  }));
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  return wave_reduce64(v, ~0ull, [](unsigned long long a, unsigned long long b) { return b < a ? b : a; });
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  return wave_reduce64(v, 0ull, [](unsigned long long a, unsigned long long b) { return b > a ? b : a; });
}

__device__ __forceinline__ int wave_or(int v) {
  return (int)wave_reduce64((unsigned)v, 0ull, [](unsigned long long a, unsigned long long b) { return a | b; });
}

// Inclusive prefix sum over the lanes of a wave, exact for integers: within each row
// the shifted copies by 1, 2 and 3 lanes, then the partial sums shifted by 4 (into
// the upper three banks of 4 lanes) and by 8 (into the upper two), then the row
// totals by the broadcasts of lanes 15 and 31.  The whole wave must be active.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
  unsigned t = v + (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);             // row_shr:2
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x113, 0xF, 0xF, false);             // row_shr:3
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)t, 0x114, 0xF, 0xE, false);             // row_shr:4
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)t, 0x118, 0xF, 0xC, false);             // row_shr:8
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)t, kDppBcast15, 0xA, 0xF, false);
  t += (unsigned)__builtin_amdgcn_update_dpp(0, (int)t, kDppBcast31, 0xC, 0xF, false);
  return t;
}

// Reduction of one BlockPartial over groups of `group` threads (a multiple of 64):
// lanes by butterfly, then the group's waves in index order; the result is valid
// in the first thread of each group.  Every thread of the block must call it.
// With group = blockDim.x this is the block-wide reduction; the batched kernel
// uses groups to reproduce the blocks of the single-system kernels exactly.
// used: the group's waves that can hold data (the rest hold zero partials, whose fold
// changes nothing: no partial is -0.0, since every sum starts from +0.0)
__device__ void group_reduce(BlockPartial &v, BlockPartial *s_waves, int group, int used = 64) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wpg = min(group >> 6, used);
  v.pe = wave_sum(v.pe);
  v.w = wave_sum(v.w);
  v.ke_half = wave_sum(v.ke_half);
  v.ke_int = wave_sum(v.ke_int);
  v.disp2 = wave_max(v.disp2);
  v.t0 = wave_min_u64(v.t0);
  v.t1 = wave_max_u64(v.t1);
  v.nonfinite = wave_or(v.nonfinite);
  if (lane == 0) s_waves[wv] = v;
  __syncthreads();
  if ((threadIdx.x % group) == 0) {
    const int w0 = wv;  // first wave of this group
    BlockPartial a = s_waves[w0];
    for (int k = 1; k < wpg; ++k) {
      const BlockPartial &q = s_waves[w0 + k];
      a.pe += q.pe;
      a.w += q.w;
      a.ke_half += q.ke_half;
      a.ke_int += q.ke_int;
      a.disp2 = fmax(a.disp2, q.disp2);
      a.nonfinite |= q.nonfinite;
      a.t0 = q.t0 < a.t0 ? q.t0 : a.t0;
      a.t1 = q.t1 > a.t1 ? q.t1 : a.t1;
    }
    v = a;
  }
}

__device__ __forceinline__ void block_reduce(BlockPartial &v, BlockPartial *s_waves) {
  group_reduce(v, s_waves, (int)blockDim.x);
}

__device__ __forceinline__ BlockPartial zero_partial() {
  BlockPartial a;
  a.pe = a.w = a.ke_half = a.ke_int = a.disp2 = 0.0;
  a.nonfinite = 0;
  a.pad = 0;
  a.t0 = ~0ull;
  a.t1 = 0ull;
  return a;
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

// Per-block totals of a list build, one device-scope atomic each: entries kept,
// the longest list (before capping) and the overflow flag.  Every thread of the
// block calls it once.
__device__ void list_tally(int cnt, int longest, int nmax, Control *ctl) {
  __shared__ int s_sum[16], s_max[16];
  int v = cnt, m = longest;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_xor(v, o, 64);
    m = max(m, __shfl_xor(m, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    s_sum[threadIdx.x >> 6] = v;
    s_max[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    int mx = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      tot += s_sum[k];
      mx = max(mx, s_max[k]);
    }
    atomicAdd((unsigned long long *)&ctl->list_entries, (unsigned long long)tot);
    atomicMax(&ctl->max_nbrs, mx);
    if (mx > nmax) atomicOr(&ctl->error, 2);
  }
}

// Copy the sorted arrays of slot t into place and record its build position.
__device__ __forceinline__ void place_sorted(const SysPtrs &p, int cur, int t, const float4 r) {
  p.pos[cur][t] = r;
  p.last[t] = r;
  p.vel[t] = p.t_vel[t];
  p.img[t] = p.t_img[t];
  if (p.kahan) p.kahan[t] = p.t_kahan[t];
  if (p.pos64) {
    p.pos64[3 * t] = p.t_pos64[3 * t];
    p.pos64[3 * t + 1] = p.t_pos64[3 * t + 1];
    p.pos64[3 * t + 2] = p.t_pos64[3 * t + 2];
  }
}

// ---------------------------------------------------------------- multi-kernel sort (large systems)

__device__ __forceinline__ void begin_build(Control *ctl) {
  ctl->max_nbrs = 0;
  ctl->list_entries = 0;
  ctl->n_rebuilds += 1;
}

// All-pairs lists keep the particle order between builds; with sort_every = k > 0
// the particles are spatially sorted again before builds 0, k, 2k, ... (the
// periodic re-sort of the paper's n2 method, appendix step 5), counted by the builds
// so far.
__device__ __forceinline__ bool resort_due(const SysConst &c, long long builds) {
  return c.sort_every > 0 && (builds % c.sort_every) == 0;
}

// The counting sort of large systems (section 7 steps 1-3) in four phases, each a
// grid-wide pass over particles or cells: bin, scan, scatter, gather.  The launch
// chain runs them as four kernels; the persistent kernel runs the same functions
// with a grid barrier between phases.  Thread ranges: a workgroup of blockDim.x
// threads starts at particle base and steps by stride.

// Phase 1: cell of every particle, its arrival slot in the cell, and the particle
// count of every tile of 2^shift cells (lanes of a wave that fall in the same tile
// add to it once).
__device__ void sort_bin(const SysConst &c, const SysPtrs &p, int cur, int base, int stride) {
  const int shift = scan_tile_shift(c.ncell);
  const int lane = threadIdx.x & 63;
  for (int s0 = base; s0 < c.n; s0 += stride) {  // uniform over the workgroup
    const int s = s0 + threadIdx.x;
    const bool act = s < c.n;
    unsigned tile = 0u;
    if (act) {
      const float4 r = p.pos[cur][s];
      int cx, cy, cz;
      cell_coords(r, c, cx, cy, cz);
      const unsigned cell = (unsigned)((cz * c.nc[1] + cy) * c.nc[0] + cx);
      p.cell_of[s] = cell;
      p.slot_in_cell[s] = atomicAdd(&p.cell_count[cell], 1u);
      tile = cell >> shift;
    }
    unsigned long long pend = __ballot(act);
    while (pend) {
      const int lead = __ffsll((long long)pend) - 1;
      const unsigned lt = (unsigned)__builtin_amdgcn_readlane((int)tile, lead);
      const unsigned long long same = __ballot(act && tile == lt);
      if (lane == lead) atomicAdd(&p.tile_count[lt], (unsigned)__popcll(same));
      pend &= ~same;
    }
  }
}

// Phase 2: exclusive scan of the cell histogram into cell_start for tile b, by the
// calling workgroup: the counts of the tiles before b, then the tile 4 cells per
// thread at a time.  The histogram is cleared for the next build (the tile counts
// are cleared in phase 3).  s_w: 16 words of LDS.
__device__ void sort_scan_tile(const SysConst &c, const SysPtrs &p, int b, unsigned *s_w) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  const int shift = scan_tile_shift(c.ncell);
  unsigned pre = 0;
  for (int k = t; k < b; k += blockDim.x) pre += p.tile_count[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
  if (lane == 0) s_w[wv] = pre;
  __syncthreads();
  unsigned carry = 0;
  for (int k = 0; k < nw; ++k) carry += s_w[k];
  __syncthreads();
  const int beg = b << shift, end = min(c.ncell, (b + 1) << shift);
  for (int base = beg; base < end; base += 4 * (int)blockDim.x) {
    const int i0 = base + 4 * t;
    unsigned v[4];
    if (i0 + 3 < end) {
      const uint4 q = *reinterpret_cast<const uint4 *>(p.cell_count + i0);
      v[0] = q.x;
      v[1] = q.y;
      v[2] = q.z;
      v[3] = q.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = i0 + k < end ? p.cell_count[i0 + k] : 0u;
    }
    const unsigned sum = v[0] + v[1] + v[2] + v[3];
    unsigned x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    unsigned wbase = 0, total = 0;
    for (int k = 0; k < nw; ++k) {
      if (k < wv) wbase += s_w[k];
      total += s_w[k];
    }
    unsigned e = carry + wbase + x - sum;
    if (i0 + 3 < end) {
      uint4 o4;
      o4.x = e;
      o4.y = e + v[0];
      o4.z = e + v[0] + v[1];
      o4.w = e + v[0] + v[1] + v[2];
      *reinterpret_cast<uint4 *>(p.cell_start + i0) = o4;
      *reinterpret_cast<uint4 *>(p.cell_count + i0) = make_uint4(0u, 0u, 0u, 0u);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i0 + k < end) {
          p.cell_start[i0 + k] = e;
          p.cell_count[i0 + k] = 0u;
        }
        e += v[k];
      }
    }
    carry += total;
    __syncthreads();  // s_w is rewritten by the next chunk
  }
  if (b == scan_tiles(c.ncell) - 1 && t == 0) p.cell_start[c.ncell] = carry;
}

// Phase 3: every particle's arrival slot in its cell's range (perm_tmp); the tile
// counts are cleared for the next build by the threads of clear_tiles.
__device__ void sort_scatter(const SysConst &c, const SysPtrs &p, int first, int stride, bool clear_tiles) {
  if (clear_tiles)
    for (int k = threadIdx.x; k < scan_tiles(c.ncell); k += blockDim.x) p.tile_count[k] = 0u;
  for (int s = first; s < c.n; s += stride) p.perm_tmp[p.cell_start[p.cell_of[s]] + p.slot_in_cell[s]] = (unsigned)s;
}

// Phase 4: deterministic rank by particle id inside each cell, and the gather of
// every per-particle array to its sorted slot in the t_* arrays.
__device__ void sort_gather(const SysConst &c, const SysPtrs &p, int cur, int first, int stride) {
  for (int s = first; s < c.n; s += stride) {
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
}

__global__ __launch_bounds__(256) void k_bin(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  sort_bin(c, p, cur, blockIdx.x * blockDim.x, gridDim.x * blockDim.x);
}

// One workgroup per tile of cells.
__global__ __launch_bounds__(256) void k_scan(SysConst c, SysPtrs p) {
  if (p.ctl->rebuild == 0) return;
  __shared__ unsigned s_w[16];
  if (blockIdx.x == 0 && threadIdx.x == 0) begin_build(p.ctl);
  sort_scan_tile(c, p, blockIdx.x, s_w);
}

__global__ __launch_bounds__(256) void k_scatter(SysConst c, SysPtrs p) {
  if (p.ctl->rebuild == 0) return;
  sort_scatter(c, p, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, blockIdx.x == 0);
}

__global__ __launch_bounds__(256) void k_gather(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  sort_gather(c, p, cur, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// ---------------------------------------------------------------- one-workgroup sort (small systems)

constexpr int kSmallN = 8192;
constexpr int kSmallCells = 8192;

// The whole spatial sort of a small system by the calling workgroup, in LDS: cell
// histogram with LDS atomics, exclusive scan (also written to cell_start), the
// particle ids placed by arrival order in their cell, a deterministic rank by
// particle id inside each cell, and the gather of every per-particle array to its
// sorted slot in the t_* arrays (section 7 steps 1-3).  Every thread of the block
// must call it.
template <int THREADS>
__device__ void sort_small_block(const SysConst &c, const SysPtrs &p, int cur, unsigned *s_cnt, int *s_id) {
  __shared__ unsigned s_w[16];
  __shared__ unsigned s_carry;
  constexpr int PER = kSmallN / THREADS;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nthr >> 6;
  const int ncell = c.ncell;
  for (int k = tid; k <= ncell; k += nthr) s_cnt[k] = 0u;
  if (tid == 0) {
    s_carry = 0u;
    begin_build(p.ctl);
    p.ctl->resorted = 1;
  }
  unsigned my_cell[PER], my_slot[PER];
  int my_id[PER];
  float4 my_pos[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int sidx = tid + m * nthr;
    my_cell[m] = 0u;
    my_slot[m] = 0u;
    my_id[m] = 0;
    my_pos[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (sidx < c.n) {
      my_pos[m] = p.pos[cur][sidx];
      my_id[m] = p.img[sidx].w;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int sidx = tid + m * nthr;
    if (sidx < c.n) {
      int cx, cy, cz;
      cell_coords(my_pos[m], c, cx, cy, cz);
      my_cell[m] = (unsigned)((cz * c.nc[1] + cy) * c.nc[0] + cx);
      my_slot[m] = atomicAdd(&s_cnt[my_cell[m]], 1u);
    }
  }
  __syncthreads();
  for (int base = 0; base <= ncell; base += nthr) {
    const int idx = base + tid;
    const unsigned v = idx <= ncell ? s_cnt[idx] : 0u;
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
    if (idx <= ncell) {
      const unsigned e = s_carry + wbase + x - v;
      s_cnt[idx] = e;
      p.cell_start[idx] = e;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned tot = 0;
      for (int k = 0; k < nw; ++k) tot += s_w[k];
      s_carry += tot;
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int sidx = tid + m * nthr;
    if (sidx < c.n) s_id[s_cnt[my_cell[m]] + my_slot[m]] = my_id[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int sidx = tid + m * nthr;
    if (sidx < c.n) {
      const unsigned beg = s_cnt[my_cell[m]], end = s_cnt[my_cell[m] + 1];
      unsigned rank = 0;
      for (unsigned q = beg; q < end; ++q) rank += (s_id[q] < my_id[m]) ? 1u : 0u;
      const unsigned dst = beg + rank;
      p.t_pos[dst] = my_pos[m];
      p.t_vel[dst] = p.vel[sidx];
      p.t_img[dst] = p.img[sidx];
      if (p.pos64) {
        p.t_pos64[3 * dst] = p.pos64[3 * sidx];
        p.t_pos64[3 * dst + 1] = p.pos64[3 * sidx + 1];
        p.t_pos64[3 * dst + 2] = p.pos64[3 * sidx + 2];
      }
      if (p.kahan) p.t_kahan[dst] = p.kahan[sidx];
    }
  }
}

// Spatial sort requested from the host (start of a run, new state or parameters).
__global__ __launch_bounds__(1024) void k_sort_small(SysConst c, SysPtrs p, int cur) {
  __shared__ unsigned s_cnt[kSmallCells + 1];
  __shared__ int s_id[kSmallN];
  __shared__ int s_due;
  if (p.ctl->rebuild == 0) return;
  if (c.list_kind == 4) {  // all-pairs lists sort only when a periodic re-sort is due
    if (threadIdx.x == 0) s_due = resort_due(c, p.ctl->n_rebuilds) ? 1 : 0;
    __syncthreads();
    if (!s_due) {
      if (threadIdx.x == 0) {
        begin_build(p.ctl);
        p.ctl->resorted = 0;
      }
      return;
    }
  }
  sort_small_block<1024>(c, p, cur, s_cnt, s_id);
}

bool small_sort_fits(int n, int ncell) { return n <= kSmallN && ncell <= kSmallCells; }

// ---------------------------------------------------------------- list builds

constexpr int kWaveCand = 1024;  // candidates per window of the wave builder
constexpr int kListChunks = 4;   // 64-candidate chunks whose loads are in flight together

// The stencil of cell (cx, cy, cz) as runs of sorted slots: 5x5x5 cells (every cell
// along an axis with fewer than 5), cut into rows of consecutive x cells; as
// particles are sorted by cell index, each row is one or two contiguous slot runs.
// Lane s of the calling wave gets run s (row s / 2; the second run of a row only
// when its x window wraps round the box) in the order of the rows, its offset excl
// in the concatenated candidate sequence and the sequence length total.
__device__ __forceinline__ void stencil_runs(const SysConst &c, int cx, int cy, int cz, const unsigned *cstart,
                                             unsigned &run_start, unsigned &run_len, unsigned &excl,
                                             unsigned &total) {
  const int lane = threadIdx.x & 63;
  const int nx = c.nc[0], ny = c.nc[1], nz = c.nc[2];
  const bool fy = c.full_axis & 2, fz = c.full_axis & 4;
  const int ny_eff = fy ? ny : 5, nz_eff = fz ? nz : 5;
  int a0, a1, b0, b1;
  row_runs(cx, nx, c.full_axis & 1, a0, a1, b0, b1);
  run_start = 0;
  run_len = 0;
  const int row = lane >> 1;
  if (row < ny_eff * nz_eff) {
    const int oy = row % ny_eff, oz = row / ny_eff;
    const int yy = fy ? oy : (cy + oy - 2 + ny) % ny;
    const int zz = fz ? oz : (cz + oz - 2 + nz) % nz;
    const int rowbase = (zz * ny + yy) * nx;
    const int x0 = (lane & 1) ? b0 : a0, x1 = (lane & 1) ? b1 : a1;
    if (x1 >= x0) {
      // clamped to [0, n]: a run never reaches outside the sorted arrays
      const unsigned s1 = min(cstart[rowbase + x1 + 1], (unsigned)c.n);
      const unsigned s0 = min(cstart[rowbase + x0], s1);
      run_start = s0;
      run_len = s1 - s0;
    }
  }
  const unsigned incl = wave_incl_scan(run_len);
  excl = incl - run_len;
  total = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
}

// Verlet list of particle t (sorted slot), one wave per particle; for small systems,
// where one thread per particle (section 7) leaves the chip idle and every thread
// waits on a long chain of dependent loads.  The 5x5x5 stencil (every cell along
// an axis with fewer than 5 cells) is cut into rows of consecutive x cells; as
// particles are sorted by cell index, each row is one or two contiguous slot runs.
// Lane s loads the bounds of run s, a wave prefix sum gives each run's offset in
// the candidate sequence, the runs are expanded into LDS, and the candidates are
// tested 64 at a time; a ballot compacts the hits in candidate order, so the
// list order is deterministic (stencil row order, then slot order).  cand is the
// calling wave's LDS window of kWaveCand entries; tpos and cstart are the sorted
// positions and the cell starts (in device memory, or copies in LDS); PLACE: also
// copy slot t's sorted data into place.  Returns the number of entries kept (all
// lanes) and raises longest to the list length before capping.
template <bool PLACE>
__device__ int list_wave_one(const SysConst &c, const SysPtrs &p, int cur, int t, unsigned *cand,
                             const float *s_cs2, const float4 *tpos, const unsigned *cstart, int &longest) {
  const int lane = threadIdx.x & 63;
  const float4 r = tpos[t];
  if (PLACE && lane == 0) place_sorted(p, cur, t, r);
  const int ti = ptype(r);
  int cx, cy, cz;
  cell_coords(r, c, cx, cy, cz);
  unsigned run_start, run_len, excl, total;
  stencil_runs(c, cx, cy, cz, cstart, run_start, run_len, excl, total);
  const int nmax = c.n_max;
  int count = 0;
  for (unsigned wbase = 0; wbase < total; wbase += kWaveCand) {
    const unsigned wend = min(total, wbase + (unsigned)kWaveCand);
    // expand this lane's run into the window
    const unsigned q0 = max(excl, wbase), q1 = min(excl + run_len, wend);
    for (unsigned q = q0; q < q1; ++q) cand[q - wbase] = run_start + (q - excl);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const unsigned wlen = wend - wbase;
    for (unsigned base = 0; base < wlen; base += 64u * kListChunks) {
      unsigned u[kListChunks];
      float4 q[kListChunks];
#pragma unroll
      for (int cb = 0; cb < kListChunks; ++cb) {
        const unsigned qi = base + 64u * cb + (unsigned)lane;
        u[cb] = qi < wlen ? cand[qi] : (unsigned)t;
        q[cb] = tpos[u[cb]];
      }
#pragma unroll
      for (int cb = 0; cb < kListChunks; ++cb) {
        bool hit = false;
        if ((int)u[cb] != t) {
          float dx, dy, dz;
          const float r2 = dist2(r, q[cb], c, dx, dy, dz);
          hit = r2 < s_cs2[ti * c.ntypes + ptype(q[cb])];
        }
        const unsigned long long mask = __ballot(hit);
        const int k = count + __popcll(mask & ((1ull << lane) - 1ull));
        if (hit && k < nmax) p.nbl[nbl_addr(t, k, c.tp, c.nvp)] = (int)u[cb];
        count += __popcll(mask);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const int kept = min(count, nmax);
  if (lane == 0) p.nnb[t] = kept;
  longest = max(longest, count);  // the caller reports the longest list and overflow
  return kept;
}

// Verlet list of particle i against every particle of the system in index order,
// by the calling wave: the paper's O(N^2) builder for small systems (section 6),
// which needs no cells and no spatial sort.  Candidates are taken 64 per chunk,
// kListChunks chunks in flight; a ballot compacts the hits in index order.  pos:
// the positions of the step (in LDS or device memory).  Also records the position
// of the build, the reference of the displacement test.  Returns the entries kept
// (all lanes) and raises longest to the list length before capping.
__device__ int list_allpairs_one(const SysConst &c, const SysPtrs &p, int i, const float *s_cs2,
                                 const float4 *pos, int &longest) {
  const int lane = threadIdx.x & 63;
  const float4 r = pos[i];
  if (lane == 0) p.last[i] = r;
  const int ti = ptype(r);
  const int nmax = c.n_max;
  int count = 0;
  for (int base = 0; base < c.n; base += 64 * kListChunks) {
    int jj[kListChunks];
    float4 q[kListChunks];
#pragma unroll
    for (int cb = 0; cb < kListChunks; ++cb) {
      jj[cb] = base + 64 * cb + lane;
      q[cb] = pos[jj[cb] < c.n ? jj[cb] : i];
    }
#pragma unroll
    for (int cb = 0; cb < kListChunks; ++cb) {
      bool hit = false;
      if (jj[cb] < c.n && jj[cb] != i) {
        float dx, dy, dz;
        const float r2 = dist2(r, q[cb], c, dx, dy, dz);
        hit = r2 < s_cs2[ti * c.ntypes + ptype(q[cb])];
      }
      const unsigned long long mask = __ballot(hit);
      const int k = count + __popcll(mask & ((1ull << lane) - 1ull));
      if (hit && k < nmax) p.nbl[nbl_addr(i, k, c.tp, c.nvp)] = jj[cb];
      count += __popcll(mask);
    }
  }
  const int kept = min(count, nmax);
  if (lane == 0) p.nnb[i] = kept;
  longest = max(longest, count);
  return kept;
}

// All-pairs lists for the launch chain, one wave per particle, four per block; the
// particles keep their order unless a periodic re-sort ran before this build.
__global__ __launch_bounds__(256) void k_list_allpairs(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  if (threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
  // after a periodic re-sort the candidates come from the sorted copy, and each wave
  // moves its own particle's slot into place
  const bool resorted = p.ctl->resorted != 0;
  const float4 *src = resorted ? p.t_pos : p.pos[cur];
  int kept = 0, longest = 0;
  if (t < c.n) {  // uniform across the wave
    if (resorted && lane == 0) place_sorted(p, cur, t, src[t]);
    const int k = list_allpairs_one(c, p, t, s_cs2, src, longest);
    if (lane == 0) kept = k;
  }
  list_tally(kept, longest, c.n_max, p.ctl);
}

// One wave per particle (list_wave_one), four particles per block.
__global__ __launch_bounds__(256) void k_list_wave(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  __shared__ unsigned s_cand[4][kWaveCand];
  if (threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
  int kept = 0, longest = 0;
  if (t < c.n) {  // uniform across the wave
    const int k = list_wave_one<true>(c, p, cur, t, s_cand[wv], s_cs2, p.t_pos, p.cell_start, longest);
    if (lane == 0) kept = k;
  }
  list_tally(kept, longest, c.n_max, p.ctl);  // every thread of the block reaches this barrier once
}

constexpr int kThreadBatch = 10;  // candidate positions in flight per thread (measured best of 8-24)
constexpr int kRing = 32;         // list slots per lane staged in LDS

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Verlet list, one thread per particle (section 7), for large systems where there
// are enough particles to fill the chip.  Candidates of one stencil row are loaded
// kThreadBatch at a time, and the cell bounds of the next row are loaded while the
// current row is tested, so that a row costs about one memory round trip.  Same
// candidate order, hence the same list, as the wave builder.
//
// The list is column-major, so the lanes of a wave write one contiguous span per
// slot only when they write the same slot together; each lane finds its entries at
// its own pace, so entries are first staged in a per-wave ring of kRing slots in
// LDS, and every slot that all lanes of the wave have passed is written out as one
// span.  A lane that runs kRing slots ahead of the slowest lane writes its later
// entries directly.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_list_thread(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  __shared__ int s_ring[4][kRing][64];
  if (threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  int(*ring)[64] = s_ring[threadIdx.x >> 6];
  const int nmax = c.n_max;
  const int nx = c.nc[0], ny = c.nc[1], nz = c.nc[2];
  const bool fy = c.full_axis & 2, fz = c.full_axis & 4;
  const int ny_eff = fy ? ny : 5, nz_eff = fz ? nz : 5, nrows = ny_eff * nz_eff;
  const unsigned nu = (unsigned)c.n;
  int kept_sum = 0, longest = 0;
  for (int t0 = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x; t0 < c.n; t0 += gridDim.x * blockDim.x) {
    const int t = t0 + threadIdx.x;  // the loop is uniform over the block; lanes past n idle
    const bool act = t < c.n;
    const float4 r = p.t_pos[act ? t : t0];
    if (act) place_sorted(p, cur, t, r);
    const int ti = ptype(r);
    int cx, cy, cz;
    cell_coords(r, c, cx, cy, cz);
    int a0, a1, b0, b1;
    row_runs(cx, nx, c.full_axis & 1, a0, a1, b0, b1);
    const bool two = b1 >= b0;
    auto row_base = [&](int rr) {
      const int oz = rr / ny_eff, oy = rr - oz * ny_eff;
      const int zz = fz ? oz : (cz + oz - 2 + nz) % nz;
      const int yy = fy ? oy : (cy + oy - 2 + ny) % ny;
      return (zz * ny + yy) * nx;
    };
    int rb = row_base(0);
    unsigned ca0 = p.cell_start[rb + a0], ca1 = p.cell_start[rb + a1 + 1], cb0 = 0, cb1 = 0;
    if (two) {
      cb0 = p.cell_start[rb + b0];
      cb1 = p.cell_start[rb + b1 + 1];
    }
    int count = 0;      // entries found by this lane
    int ring_end = 0;   // this lane's entries below it are in the ring (or written)
    bool spill = false; // this lane writes its later entries directly
    int flushed = 0;    // uniform: every lane's slots below it are written
    auto flush = [&](int upto) {
      for (int k = flushed; k < upto; ++k)
        if (act && k < ring_end && k < nmax) p.nbl[nbl_addr(t, k, c.tp, c.nvp)] = ring[k % kRing][lane];
      flushed = upto;
    };
    for (int rr = 0; rr < nrows; ++rr) {
      // runs clamped to [0, n]: they never reach outside the sorted arrays
      const unsigned sa1 = min(ca1, nu), sa0 = min(ca0, sa1);
      const unsigned sb1 = two ? min(cb1, nu) : 0u, sb0 = two ? min(cb0, sb1) : 0u;
      if (rr + 1 < nrows) {
        rb = row_base(rr + 1);
        ca0 = p.cell_start[rb + a0];
        ca1 = p.cell_start[rb + a1 + 1];
        if (two) {
          cb0 = p.cell_start[rb + b0];
          cb1 = p.cell_start[rb + b1 + 1];
        }
      }
      const unsigned la = sa1 - sa0, lt = act ? la + (sb1 - sb0) : 0u;
      for (unsigned base = 0; base < lt; base += kThreadBatch) {
        unsigned u[kThreadBatch];
        float4 q[kThreadBatch];
#pragma unroll
        for (int b = 0; b < kThreadBatch; ++b) {
          const unsigned o = base + b;
          u[b] = o < la ? sa0 + o : sb0 + (o - la);
          if (o >= lt) u[b] = (unsigned)t;  // past the row: load own slot, skipped below
          q[b] = p.t_pos[u[b]];
        }
#pragma unroll
        for (int b = 0; b < kThreadBatch; ++b) {
          if (base + b < lt && (int)u[b] != t) {
            float dx, dy, dz;
            const float r2 = dist2(r, q[b], c, dx, dy, dz);
            if (r2 < s_cs2[ti * c.ntypes + ptype(q[b])]) {
              if (!spill && count - flushed >= kRing) spill = true;
              if (spill) {
                if (count < nmax) p.nbl[nbl_addr(t, count, c.tp, c.nvp)] = (int)u[b];
              } else {
                ring[count % kRing][lane] = (int)u[b];
                ring_end = count + 1;
              }
              ++count;
            }
          }
        }
      }
      // write out the slots every lane has passed, once half the ring is in use
      if (__any(act && !spill && count - flushed >= kRing / 2))
        flush(min(wave_min_int(act && !spill ? count : 0x7fffffff), flushed + kRing));
    }
    flush(flushed + kRing);
    const int kept = act ? min(count, nmax) : 0;
    if (act) p.nnb[t] = kept;
    longest = max(longest, act ? count : 0);
    kept_sum += kept;
  }
  list_tally(kept_sum, longest, nmax, p.ctl);
}

// Row-staged list build (list mode 5): one workgroup per x-row of cells.  The
// particles of a row are consecutive sorted slots, and so is every full x-row of
// the stencil, so for each of the 25 stencil rows (in the order of the other
// builders: z offset, then y offset) the workgroup copies that row's positions and
// cell starts into LDS with coalesced loads; each thread then tests its particle
// against the candidates of its five x cells from LDS, in the same slot order as
// k_list_thread, so the lists are the same entry for entry.  The per-lane gathers
// of the thread builder (a cache line per lane and candidate batch) become one
// contiguous copy per row that every particle of the row shares.  A stencil row of
// more than kRowCap particles is read from device memory instead.
constexpr int kRowCap = 1024;    // particles of a stencil row staged in LDS
constexpr int kRowCells = 1024;  // cells per x-row the cell starts of LDS hold (nc <= 1024)

__global__ __launch_bounds__(256) void k_list_row(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  __shared__ int s_ring[4][kRing][64];
  __shared__ float4 s_row[kRowCap];
  __shared__ unsigned s_cs[kRowCells + 1];
  if (threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  const int lane = threadIdx.x & 63;
  int(*ring)[64] = s_ring[threadIdx.x >> 6];
  const int nmax = c.n_max;
  const int nx = c.nc[0], ny = c.nc[1], nz = c.nc[2];
  const bool fy = c.full_axis & 2, fz = c.full_axis & 4;
  const int ny_eff = fy ? ny : 5, nz_eff = fz ? nz : 5, nrows = ny_eff * nz_eff;
  const unsigned nu = (unsigned)c.n;
  const int row = xcd_remap(blockIdx.x, gridDim.x);  // x-row (cy, cz) of this workgroup
  const int cy = row % ny, cz = row / ny;
  const unsigned r0 = min(p.cell_start[row * nx], nu), r1 = min(p.cell_start[row * nx + nx], nu);
  int kept_sum = 0, longest = 0;
  for (unsigned t0 = r0; t0 < r1; t0 += blockDim.x) {  // uniform over the block
    const unsigned tt = t0 + threadIdx.x;
    const bool act = tt < r1;
    const int t = (int)(act ? tt : r0);
    const float4 r = p.t_pos[t];
    if (act) place_sorted(p, cur, t, r);
    const int ti = ptype(r);
    int cx, cyy, czz;
    cell_coords(r, c, cx, cyy, czz);
    int a0, a1, b0, b1;
    row_runs(cx, nx, c.full_axis & 1, a0, a1, b0, b1);
    const bool two = b1 >= b0;
    int count = 0, ring_end = 0, flushed = 0;
    bool spill = false;
    auto flush = [&](int upto) {
      for (int k = flushed; k < upto; ++k)
        if (act && k < ring_end && k < nmax) p.nbl[nbl_addr(t, k, c.tp, c.nvp)] = ring[k % kRing][lane];
      flushed = upto;
    };
    for (int rr = 0; rr < nrows; ++rr) {
      const int oz = rr / ny_eff, oy = rr - oz * ny_eff;
      const int zz = fz ? oz : (cz + oz - 2 + nz) % nz;
      const int yy = fy ? oy : (cy + oy - 2 + ny) % ny;
      const int rb = (zz * ny + yy) * nx;
      __syncthreads();  // the previous row's LDS copy is no longer read
      for (int k = threadIdx.x; k <= nx; k += blockDim.x) s_cs[k] = min(p.cell_start[rb + k], nu);
      __syncthreads();
      const unsigned q0 = s_cs[0], q1 = s_cs[nx];
      const bool staged = q1 - q0 <= (unsigned)kRowCap;
      if (staged)
        for (unsigned k = threadIdx.x; k < q1 - q0; k += blockDim.x) s_row[k] = p.t_pos[q0 + k];
      __syncthreads();
      const unsigned sa0 = s_cs[a0], sa1 = s_cs[a1 + 1];
      const unsigned sb0 = two ? s_cs[b0] : 0u, sb1 = two ? s_cs[b1 + 1] : 0u;
      const unsigned la = sa1 - sa0, lt = act ? la + (sb1 - sb0) : 0u;
      for (unsigned o = 0; o < lt; ++o) {
        const unsigned u = o < la ? sa0 + o : sb0 + (o - la);
        if ((int)u == t) continue;
        const float4 q = staged ? s_row[u - q0] : p.t_pos[u];
        float dx, dy, dz;
        const float r2 = dist2(r, q, c, dx, dy, dz);
        if (r2 < s_cs2[ti * c.ntypes + ptype(q)]) {
          if (!spill && count - flushed >= kRing) spill = true;
          if (spill) {
            if (count < nmax) p.nbl[nbl_addr(t, count, c.tp, c.nvp)] = (int)u;
          } else {
            ring[count % kRing][lane] = (int)u;
            ring_end = count + 1;
          }
          ++count;
        }
      }
      // write out the slots every lane has passed, once half the ring is in use
      if (__any(act && !spill && count - flushed >= kRing / 2))
        flush(min(wave_min_int(act && !spill ? count : 0x7fffffff), flushed + kRing));
    }
    flush(flushed + kRing);
    const int kept = act ? min(count, nmax) : 0;
    if (act) p.nnb[t] = kept;
    longest = max(longest, act ? count : 0);
    kept_sum += kept;
  }
  list_tally(kept_sum, longest, nmax, p.ctl);
}

constexpr int kCellChunks = 8;  // 64-candidate chunks held in registers (one window)
constexpr int kCellWindow = 64 * kCellChunks;

// Verlet lists of the particles in sorted slots [i0, i1) of cell (cx, cy, cz), by the
// calling wave.  Every particle of a cell has the same stencil (section 7), hence the
// same candidates in the same order, so the wave loads them once, kCellWindow at a
// time (64 per chunk from contiguous slot runs), and tests each particle against
// them; a ballot compacts the hits in candidate order, so the lists equal those of
// the particle-by-particle builders entry for entry.  cand: kCellWindow entries of
// the wave's LDS; cnt[l]: entries found so far for particle i0 + l (LDS, the caller
// clears it); sink(i, k, j) stores entry k of particle i (called by the hit lanes).
template <class Sink>
__device__ void list_cell_particles(const SysConst &c, const SysPtrs &p, int cx, int cy, int cz, int i0, int i1,
                                    unsigned *cand, int *cnt, const float *s_cs2, const float4 *tpos,
                                    const unsigned *cstart, Sink sink) {
  const int lane = threadIdx.x & 63;
  unsigned run_start, run_len, excl, total;
  stencil_runs(c, cx, cy, cz, cstart, run_start, run_len, excl, total);
  for (unsigned wbase = 0; wbase < total; wbase += kCellWindow) {
    const unsigned wend = min(total, wbase + (unsigned)kCellWindow), wlen = wend - wbase;
    const unsigned q0 = max(excl, wbase), q1 = min(excl + run_len, wend);
    for (unsigned q = q0; q < q1; ++q) cand[q - wbase] = run_start + (q - excl);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned u[kCellChunks];
    float4 q[kCellChunks];
#pragma unroll
    for (int cb = 0; cb < kCellChunks; ++cb) {
      const unsigned qi = 64u * cb + (unsigned)lane;
      u[cb] = qi < wlen ? cand[qi] : (unsigned)i0;
      if (64u * cb < wlen) q[cb] = tpos[u[cb]];
    }
    for (int i = i0; i < i1; ++i) {
      const float4 pi = tpos[i];
      const int ti = ptype(pi);
      int count = cnt[i - i0];
#pragma unroll
      for (int cb = 0; cb < kCellChunks; ++cb) {
        if (64u * cb < wlen) {  // uniform over the wave
          bool hit = false;
          if (64u * cb + (unsigned)lane < wlen && (int)u[cb] != i) {
            float dx, dy, dz;
            const float r2 = dist2(pi, q[cb], c, dx, dy, dz);
            hit = r2 < s_cs2[ti * c.ntypes + ptype(q[cb])];
          }
          const unsigned long long mask = __ballot(hit);
          if (hit) sink(i, count + __popcll(mask & ((1ull << lane) - 1ull)), (int)u[cb]);
          count += __popcll(mask);
        }
      }
      if (lane == 0) cnt[i - i0] = count;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

constexpr int kCellSlots = 32;   // sorted slots per workgroup of the cell builder
constexpr int kCellStage = 128;  // list entries per particle staged in LDS

// Verlet lists, one wave per cell (list_cell_particles), for the launch chain.  A
// workgroup of two waves takes kCellSlots consecutive sorted slots, split into runs
// of one cell (a cell that straddles two workgroups is handled by both, each for its
// own slots).  The lists are staged in LDS as [particle][entry] and then written out
// by the workgroup in address order, so each entry index of the column-major list is
// one contiguous span; entries past kCellStage are written directly.
__global__ __launch_bounds__(128) void k_list_cell(SysConst c, SysPtrs p, int cur) {
  if (p.ctl->rebuild == 0) return;
  __shared__ float s_cs2[kMaxPairs];
  __shared__ int s_list[kCellSlots][kCellStage + 1];  // +1: entries of one particle fall in distinct banks
  __shared__ unsigned s_cand[2][kCellWindow];
  __shared__ int s_cnt[kCellSlots];
  __shared__ int s_seg[kCellSlots + 1];
  __shared__ int s_nseg;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int T0 = xcd_remap(blockIdx.x, gridDim.x) * kCellSlots;
  const int m = min(kCellSlots, c.n - T0);  // slots of this workgroup, >= 1
  const int nmax = c.n_max;
  if (tid < kMaxPairs) s_cs2[tid] = c.pt.cs2[tid];
  if (wv == 0) {
    // runs of slots in one cell: a segment starts where the cell index changes
    int cell = -1;
    if (lane < m) {
      const float4 r = p.t_pos[T0 + lane];
      place_sorted(p, cur, T0 + lane, r);
      int cx, cy, cz;
      cell_coords(r, c, cx, cy, cz);
      cell = (cz * c.nc[1] + cy) * c.nc[0] + cx;
      s_cnt[lane] = 0;
    }
    const int prev = __shfl_up(cell, 1, 64);
    const bool head = lane < m && (lane == 0 || prev != cell);
    const unsigned long long hm = __ballot(head);
    if (head) s_seg[__popcll(hm & ((1ull << lane) - 1ull))] = lane;
    if (lane == 0) {
      s_nseg = __popcll(hm);
      s_seg[__popcll(hm)] = m;
    }
  }
  __syncthreads();
  const int nseg = s_nseg;
  auto stage = [&](int i, int k, int j) {
    if (k < kCellStage)
      s_list[i - T0][k] = j;
    else if (k < nmax)
      p.nbl[nbl_addr(i, k, c.tp, c.nvp)] = j;
  };
  for (int sg = wv; sg < nseg; sg += 2) {
    const int l0 = s_seg[sg], l1 = s_seg[sg + 1];
    int cx, cy, cz;
    cell_coords(p.t_pos[T0 + l0], c, cx, cy, cz);
    list_cell_particles(c, p, cx, cy, cz, T0 + l0, T0 + l1, s_cand[wv], s_cnt + l0, s_cs2, p.t_pos, p.cell_start,
                        stage);
  }
  __syncthreads();
  // write-out in address order: groups of tp entries of consecutive particles are
  // contiguous in the tp-interleaved column-major list
  int kmax = 0;
  for (int l = 0; l < m; ++l) kmax = max(kmax, s_cnt[l]);
  const int tp = c.tp;
  const int kst = min(min(kmax, nmax), kCellStage);
  const int span = kCellSlots * tp;  // elements of one group of tp entries
  const int groups = (kst + tp - 1) / tp;
  for (int j = tid; j < groups * span; j += blockDim.x) {
    const int g = j / span, rr = j - g * span, l = rr / tp, k = g * tp + (rr - l * tp);
    if (l < m && k < kst && k < s_cnt[l])
      p.nbl[(long long)g * ((long long)c.nvp * tp) + (long long)(T0 + l) * tp + (rr - l * tp)] = s_list[l][k];
  }
  int kept = 0, longest = 0;
  if (tid < m) {
    longest = s_cnt[tid];
    kept = min(longest, nmax);
    p.nnb[T0 + tid] = kept;
  }
  list_tally(kept, longest, nmax, p.ctl);
}

// ---------------------------------------------------------------- force only

template <int TP, int METHOD>
__global__ __launch_bounds__(1024) void k_force(SysConst c, SysPtrs p, int cur) {
  __shared__ SharedPairs sp;
  __shared__ BlockPartial s_waves[16];
  const unsigned long long tstart = wall_clock64();
  stage_pairs(sp, c);
  __syncthreads();
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int gt = lb * blockDim.x + threadIdx.x;
  const int i = gt / TP, t = gt % TP;
  const bool active = i < c.n;
  const float4 *pos = p.pos[cur];
  float fx = 0.f, fy = 0.f, fz = 0.f, u = 0.f, w = 0.f;
  float4 vo = make_float4(0.f, 0.f, 0.f, 0.f), pi = vo;
  if (active) {
    pi = pos[i];
    if (t == 0) vo = p.vel[i];
    force_lane<TP, METHOD, StepBatch<TP>::value, true>(i, t, pi, pos, (const int *)p.nbl, (const int *)p.nnb, sp, c, fx, fy,
                                             fz, u, w);
  }
  fx = lane_sum<TP>(fx);
  fy = lane_sum<TP>(fy);
  fz = lane_sum<TP>(fz);
  u = lane_sum<TP>(u);
  w = lane_sum<TP>(w);
  BlockPartial v = zero_partial();
  if (active && t == 0) {
    p.force[i] = make_float4(fx, fy, fz, 0.5f * u);
    p.wpart[i] = (float)((double)w / 6.0);
    v.pe = 0.5 * (double)u;
    v.w = (double)w / 6.0;
    const double dvx = vo.x, dvy = vo.y, dvz = vo.z;
    v.ke_half = 0.5 * c.mass[ptype(pi)] * (dvx * dvx + dvy * dvy + dvz * dvz);
    v.nonfinite = finite3(fx, fy, fz) ? 0 : 1;
  }
  v.t0 = tstart;
  v.t1 = wall_clock64();
  block_reduce(v, s_waves);
  if (threadIdx.x == 0) {
    p.part[lb] = v;
    if (blockIdx.x == 0) p.ctl->rebuild = 0;  // the list in use is now current
  }
}

// A store that writes through the L2 to memory: agent-scope relaxed atomic stores of
// its 8-byte words (the XCDs' L2s are not coherent with each other).  Once the
// storing wave's vmcnt has drained the words are visible to loads from any XCD
// that miss their own L2, with no write-back of a whole L2.
template <class T>
__device__ __forceinline__ void store_through(T *dst, const T &v) {
  static_assert(sizeof(T) % 8 == 0, "whole 8-byte words");
  unsigned long long w[sizeof(T) / 8];
  __builtin_memcpy(w, &v, sizeof(T));
  unsigned long long *d = reinterpret_cast<unsigned long long *>(dst);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 8); ++k) __hip_atomic_store(d + k, w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void store_to(T *dst, const T &v, bool through) {
  if (through)
    store_through(dst, v);
  else
    *dst = v;
}

// Leapfrog / Nose-Hoover update of particle i (sorted slot) from its force, and
// its float64 contributions to the step's sums (paper section 2 integrators;
// kinetic energy at the half step for the thermostat and at the integer step for
// the thermodynamic record; largest displacement since the last list build for
// the rebuild test of section 6).
template <int PREC>
__device__ __forceinline__ void integrate_one(const SysConst &c, const SysPtrs &p, int cur, int i, const float4 pi,
                                              const float4 vo, int4 im, const float4 l0, float4 kc, double x64,
                                              double y64, double z64, double xi, float fx, float fy, float fz,
                                              float u, float w, BlockPartial &v, bool through = false) {
    // through: the arrays the end-of-step sort reads are written through the L2
    const int ti = ptype(pi);
    // v(n+1/2) = [v(n-1/2) (1 - xi dt/2) + F/m dt] / (1 + xi dt/2); a = b = 1 without thermostat
    const double hx = 0.5 * xi * c.dtd;
    const float a = (float)(1.0 - hx);
    const float ib = (float)(1.0 / (1.0 + hx));
    const float dtm = c.dt * c.inv_mass[ti];
    const float vx = __builtin_fmaf(vo.x, a, fx * dtm) * ib;
    const float vy = __builtin_fmaf(vo.y, a, fy * dtm) * ib;
    const float vz = __builtin_fmaf(vo.z, a, fz * dtm) * ib;
    store_to(&p.vel[i], make_float4(vx, vy, vz, vo.w), through);
    p.force[i] = make_float4(fx, fy, fz, 0.5f * u);
    float4 rn;
    rn.w = pi.w;
    if (PREC == 2) {  // float64 master positions
      double x = x64 + (double)vx * c.dtd;
      double y = y64 + (double)vy * c.dtd;
      double z = z64 + (double)vz * c.dtd;
      if (x >= 0.5 * c.Ld[0]) { x -= c.Ld[0]; im.x += 1; } else if (x < -0.5 * c.Ld[0]) { x += c.Ld[0]; im.x -= 1; }
      if (y >= 0.5 * c.Ld[1]) { y -= c.Ld[1]; im.y += 1; } else if (y < -0.5 * c.Ld[1]) { y += c.Ld[1]; im.y -= 1; }
      if (z >= 0.5 * c.Ld[2]) { z -= c.Ld[2]; im.z += 1; } else if (z < -0.5 * c.Ld[2]) { z += c.Ld[2]; im.z -= 1; }
      store_to(&p.pos64[3 * i], x, through);
      store_to(&p.pos64[3 * i + 1], y, through);
      store_to(&p.pos64[3 * i + 2], z, through);
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
        const float yx = vx * c.dt - kc.x, yy = vy * c.dt - kc.y, yz = vz * c.dt - kc.z;
        x = pi.x + yx;
        y = pi.y + yy;
        z = pi.z + yz;
        kc.x = (x - pi.x) - yx;
        kc.y = (y - pi.y) - yy;
        kc.z = (z - pi.z) - yz;
        store_to(&p.kahan[i], kc, through);
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
    store_to(&p.pos[cur ^ 1][i], rn, through);
    store_to(&p.img[i], im, through);
    // float64 reductions
    const double m = c.mass[ti];
    const double dvx = vx, dvy = vy, dvz = vz;
    v.ke_half = 0.5 * m * (dvx * dvx + dvy * dvy + dvz * dvz);
    const double mx = 0.5 * ((double)vo.x + dvx), my = 0.5 * ((double)vo.y + dvy), mz = 0.5 * ((double)vo.z + dvz);
    v.ke_int = 0.5 * m * (mx * mx + my * my + mz * mz);
    v.pe = 0.5 * (double)u;
    v.w = (double)w / 6.0;
    // displacement since the last build: float64 from the float32 positions
    double ddx = (double)rn.x - (double)l0.x, ddy = (double)rn.y - (double)l0.y, ddz = (double)rn.z - (double)l0.z;
    ddx -= c.Ld[0] * rint(ddx / c.Ld[0]);
    ddy -= c.Ld[1] * rint(ddy / c.Ld[1]);
    ddz -= c.Ld[2] * rint(ddz / c.Ld[2]);
    v.disp2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
    v.nonfinite = (finite3(fx, fy, fz) && finite3(rn.x, rn.y, rn.z)) ? 0 : 1;
}

// ---------------------------------------------------------------- end of step

// Nose-Hoover friction of the next step from the half-step kinetic energy.
__device__ __forceinline__ double xi_next(const SysConst &c, double xi, double ke_half) {
  const double th = 2.0 * ke_half / c.g;
  return xi + c.dtd * (th / c.T0 - 1.0) * c.inv_tau2;
}

// End of a time step, by one thread, from the fully reduced partials a: the
// thermodynamic record, the Nose-Hoover update, the step counter and the
// displacement test that sets the rebuild flag.  Returns the flag.
// The control words finish_step reads, loaded together (one memory round trip).
struct CtlView {
  double xi, xi_int;
  long long step, n_rebuilds, n_records, trace_cap;
  int max_nbrs, thermo_every;
};

__device__ __forceinline__ CtlView load_ctl(const Control *ctl) {
  CtlView v;
  v.xi = ctl->xi;
  v.xi_int = ctl->xi_int;
  v.step = ctl->step;
  v.n_rebuilds = ctl->n_rebuilds;
  v.n_records = ctl->n_records;
  v.trace_cap = ctl->trace_cap;
  v.max_nbrs = ctl->max_nbrs;
  v.thermo_every = ctl->thermo_every;
  return v;
}

// End of a time step, by one thread, from the fully reduced partials a and the
// control words v (loaded after the step's list build): the thermodynamic record,
// the Nose-Hoover update, the step counter and the displacement test that sets the
// rebuild flag.  Returns the flag.
__device__ int finish_step(const SysConst &c, const SysPtrs &p, const BlockPartial &a, const CtlView &v) {
  Control *ctl = p.ctl;
  const double xi = c.thermostat ? v.xi : 0.0;
  Thermo rec;
  rec.pe = a.pe;
  rec.ke = a.ke_int;
  rec.virial = a.w;
  rec.temperature = 2.0 * a.ke_int / c.g;
  rec.pressure = (2.0 * a.ke_int / 3.0 + a.w) / c.volume;
  rec.xi = xi;
  rec.xi_integral = v.xi_int;
  rec.h_conserved = a.ke_int + a.pe;
  if (c.thermostat && c.inv_tau2 > 0.0)
    rec.h_conserved += c.g * c.T0 * (xi * xi / (2.0 * c.inv_tau2) + v.xi_int);
  rec.ke_half = a.ke_half;
  rec.step = v.step;
  rec.n_rebuilds = v.n_rebuilds;
  rec.max_nbrs = v.max_nbrs;
  rec.reserved = 0;
  *p.thermo = rec;
  if (v.thermo_every > 0 && (v.step % v.thermo_every) == 0 && v.n_records < v.trace_cap) {
    p.trace[v.n_records] = rec;
    ctl->n_records = v.n_records + 1;
  }
  if (c.thermostat) {
    const double xn = xi_next(c, xi, a.ke_half);
    ctl->xi_int = v.xi_int + c.dtd * (xi + xn) * 0.5;
    ctl->xi = xn;
  }
  ctl->step = v.step + 1;
  if (a.t1 > a.t0) {
    ctl->prof_ticks += a.t1 - a.t0;
    ctl->prof_count += 1;
  }
  const int rebuild = (a.disp2 > c.half_skin2) ? 1 : 0;
  ctl->rebuild = rebuild;
  if (a.nonfinite) atomicOr(&ctl->error, 1);
  return rebuild;
}

// ---------------------------------------------------------------- end of step in the step kernel

// The fold of one block partial into a running sum, with the operations and order
// of k_finish and group_reduce (the device-clock stamps included).
__device__ __forceinline__ void fold_timed(BlockPartial &a, const BlockPartial &q) {
  a.pe += q.pe;
  a.w += q.w;
  a.ke_half += q.ke_half;
  a.ke_int += q.ke_int;
  a.disp2 = fmax(a.disp2, q.disp2);
  a.nonfinite |= q.nonfinite;
  a.t0 = q.t0 < a.t0 ? q.t0 : a.t0;
  a.t1 = q.t1 > a.t1 ? q.t1 : a.t1;
}

// Arrival counters of a step kernel that ends the step itself: kArriveGroups group
// counters and one top counter, each on its own 128-byte line.
constexpr unsigned kArriveGroups = 16;
constexpr unsigned kArriveStride = 32;  // unsigned words per counter line
constexpr size_t kArriveBytes = sizeof(unsigned) * kArriveStride * (kArriveGroups + 1);

// Arrival of a workgroup at the end of a step kernel that ends the step itself.
// What the last workgroup reads from the others (their block partials and, for a
// small system, the arrays its sort reads) was written through the L2
// (store_through); every wave waits for its stores to complete before its
// workgroup takes a ticket.  No L2 write-back is needed (one per workgroup would
// cost the XCD's L2 a walk each).  Tickets are taken in two levels, so that the
// workgroups that end together do not all queue on one word: workgroup b counts on
// group counter b % 16, and the last of each group on the top counter.  The
// workgroup with the last top ticket acquires at agent scope (the invalidation of
// its compute unit's L1 and of its L2 precedes, through the workgroup barrier,
// every later load of its waves) and returns true in all its threads.  Each counter
// is put back to zero by the workgroup that takes its last ticket, for the next
// launch.  Every workgroup has arrived, hence read the step's control words, before
// the last one writes them.
__device__ __forceinline__ bool arrive_last(unsigned *ctr, unsigned G, unsigned b, int *s_last) {
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = b % kArriveGroups;
    const unsigned members = G / kArriveGroups + (g < G % kArriveGroups ? 1u : 0u);
    const unsigned groups = G < kArriveGroups ? G : kArriveGroups;
    int last = 0;
    unsigned *gc = ctr + g * kArriveStride, *top = ctr + kArriveGroups * kArriveStride;
    if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == members) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == groups) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = 1;
      }
    }
    *s_last = last;
  }
  __syncthreads();
  return *s_last != 0;
}

// The reduction of k_finish<0> (1024 threads: thread t sums the block partials t,
// t + 1024, ... in order, a butterfly per wave, then thread 0 folds in order the
// waves that hold data) by a workgroup of any multiple of 64 threads, its wave v
// standing in for the waves v, v + W, ... of that workgroup.  Bitwise the result of
// k_finish; valid in thread 0.
__device__ BlockPartial finish_reduce(const BlockPartial *part, int G, BlockPartial *s_waves) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  const int used = min(16, (G + 63) / 64);
  for (int vw = wv; vw < used; vw += nw) {
    BlockPartial a = zero_partial();
    for (int b = vw * 64 + lane; b < G; b += 1024) fold_timed(a, part[b]);
    a.pe = wave_sum(a.pe);
    a.w = wave_sum(a.w);
    a.ke_half = wave_sum(a.ke_half);
    a.ke_int = wave_sum(a.ke_int);
    a.disp2 = wave_max(a.disp2);
    a.t0 = wave_min_u64(a.t0);
    a.t1 = wave_max_u64(a.t1);
    a.nonfinite = wave_or(a.nonfinite);
    if (lane == 0) s_waves[vw] = a;
  }
  __syncthreads();
  BlockPartial a = zero_partial();
  if (threadIdx.x == 0) {
    a = s_waves[0];
    for (int k = 1; k < used; ++k) fold_timed(a, s_waves[k]);
  }
  return a;
}

// Cell index of a position (the major key of the spatial sort).
__device__ __forceinline__ int cell_index(const float4 r, const SysConst &c) {
  int cx, cy, cz;
  cell_coords(r, c, cx, cy, cz);
  return (cz * c.nc[1] + cy) * c.nc[0] + cx;
}

// The spatial sort of sort_small_block (order by cell, then particle id; the same
// cell starts and gathered arrays) by a workgroup of any size, its working arrays
// in LDS only: s_cnt (ncell + 1 words) and s_id (n words).  A histogram pass, the
// exclusive scan (also written to cell_start), a placement pass that moves each
// cell's cursor past its particles (so that afterwards s_cnt[k] ends cell k), and a
// rank-and-gather pass; cells are recomputed from the positions in every pass.
// Each thread takes B particles of a pass at a time, their loads issued together
// (B / 2 in the gather pass, which loads three arrays), so that a pass over a few
// thousand particles costs one memory round trip rather than one per particle; when
// all particles fit one such batch, the placement works from registers instead
// (below).  The scan's per-wave prefix sums are DPP lane shifts.
template <int B>
__device__ void sort_small_shared(const SysConst &c, const SysPtrs &p, int cur, unsigned *s_cnt, int *s_id) {
  constexpr int BG = B > 1 ? B / 2 : 1;
  __shared__ unsigned s_w[16];
  __shared__ unsigned s_carry;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = (nthr + 63) >> 6;
  const int ncell = c.ncell, n = c.n;
  const float4 *pos = p.pos[cur];
  for (int k = tid; k <= ncell; k += nthr) s_cnt[k] = 0u;
  if (tid == 0) {
    s_carry = 0u;
    begin_build(p.ctl);
    p.ctl->resorted = 1;
  }
  __syncthreads();
  // When each thread has at most B particles (one batch), their cells, ids and slots
  // within their cells (the histogram counter before their increment) stay in
  // registers, and the placement needs neither the positions again nor a second
  // atomic: particle k goes to start(cell) + slot.  key = cell << 13 | slot (cells
  // and slots below 8192, as N <= 8192).
  const bool one = B > 1 && n <= B * nthr;
  unsigned key[B];
  int idr[B];
  // (loads past n are clamped to the last particle and their results unused, so that
  // every load is issued unconditionally)
  for (int base = tid; base < n; base += B * nthr) {
    float4 r[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int i = min(base + k * nthr, n - 1);
      r[k] = pos[i];
      if (one) idr[k] = p.img[i].w;
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (base + k * nthr < n) {
        const unsigned cell = (unsigned)cell_index(r[k], c);
        const unsigned slot = atomicAdd(&s_cnt[cell], 1u);
        if (one) key[k] = cell << 13 | slot;
      }
  }
  __syncthreads();
  for (int base = 0; base <= ncell; base += nthr) {
    const int idx = base + tid;
    const unsigned v = idx <= ncell ? s_cnt[idx] : 0u;
    const unsigned x = wave_incl_scan(v);
    if (lane == 63 || tid == nthr - 1) s_w[wv] = x;
    __syncthreads();
    unsigned wbase = 0;
    for (int k = 0; k < wv; ++k) wbase += s_w[k];
    if (idx <= ncell) {
      const unsigned e = s_carry + wbase + x - v;
      s_cnt[idx] = e;
      p.cell_start[idx] = e;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned tot = 0;
      for (int k = 0; k < nw; ++k) tot += s_w[k];
      s_carry += tot;
    }
    __syncthreads();
  }
  if (one) {
    // s_cnt holds the cell starts (and s_cnt[ncell] = n)
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (tid + k * nthr < n) s_id[s_cnt[key[k] >> 13] + (key[k] & 8191u)] = idr[k];
  } else {
    for (int base = tid; base < n; base += B * nthr) {
      float4 r[B];
      int id[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int i = min(base + k * nthr, n - 1);
        r[k] = pos[i];
        id[k] = p.img[i].w;
      }
#pragma unroll
      for (int k = 0; k < B; ++k)
        if (base + k * nthr < n) s_id[atomicAdd(&s_cnt[cell_index(r[k], c)], 1u)] = id[k];
    }
  }
  __syncthreads();
  for (int base = tid; base < n; base += BG * nthr) {
    float4 r[BG];
    raw_f4 v[BG];
    raw_i4 im[BG];
#pragma unroll
    for (int k = 0; k < BG; ++k) {
      const int i = min(base + k * nthr, n - 1);
      r[k] = pos[i];
      im[k] = reinterpret_cast<const raw_i4 *>(p.img)[i];
      v[k] = reinterpret_cast<const raw_f4 *>(p.vel)[i];
    }
#pragma unroll
    for (int k = 0; k < BG; ++k) {
      const int i = base + k * nthr;
      if (i < n) {
        const int cell = cell_index(r[k], c);
        // cell bounds: starts (one batch) or the cursors moved to the cells' ends
        const unsigned beg = one ? s_cnt[cell] : cell > 0 ? s_cnt[cell - 1] : 0u;
        const unsigned end = one ? s_cnt[cell + 1] : s_cnt[cell];
        unsigned rank = 0;
        for (unsigned q = beg; q < end; ++q) rank += (s_id[q] < im[k].w) ? 1u : 0u;
        const unsigned dst = beg + rank;
        p.t_pos[dst] = r[k];
        reinterpret_cast<raw_f4 *>(p.t_vel)[dst] = v[k];
        reinterpret_cast<raw_i4 *>(p.t_img)[dst] = im[k];
        if (p.pos64) {
          p.t_pos64[3 * dst] = p.pos64[3 * i];
          p.t_pos64[3 * dst + 1] = p.pos64[3 * i + 1];
          p.t_pos64[3 * dst + 2] = p.pos64[3 * i + 2];
        }
        if (p.kahan) p.t_kahan[dst] = p.kahan[i];
      }
    }
  }
}

// Particles per thread whose loads the end-of-step sort issues together.
constexpr int kTailSortBatch = 8;

// LDS bytes of sort_small_shared for n particles in ncell cells.
__host__ __device__ constexpr size_t tail_sort_lds(int n, int ncell) { return 4 * ((size_t)ncell + 1 + (size_t)n); }

// The end of a step in the workgroup that arrived last (arrive_last): the
// reduction, record, thermostat update and rebuild decision of k_finish<0>, and on
// a small system's step that decides a rebuild the spatial sort of the new
// positions pos[next] (dynamic LDS of tail_sort_lds bytes).
__device__ void step_tail(const SysConst &c, const SysPtrs &p, int G, int next, BlockPartial *s_waves, int *s_flag,
                          unsigned *s_dyn) {
  CtlView cv{};
  if (threadIdx.x == 0) cv = load_ctl(p.ctl);  // beside the partials: one round trip
  const BlockPartial a = finish_reduce(p.part, G, s_waves);
  if (threadIdx.x == 0) {
    s_flag[0] = finish_step(c, p, a, cv);
    s_flag[1] = resort_due(c, cv.n_rebuilds) ? 1 : 0;
  }
  __syncthreads();
  if (s_flag[0] && c.small_sort) {
    if (c.list_kind == 4 && !s_flag[1]) {  // all-pairs lists sort only when a re-sort is due
      if (threadIdx.x == 0) {
        begin_build(p.ctl);
        p.ctl->resorted = 0;
      }
    } else {
      sort_small_shared<kTailSortBatch>(c, p, next, s_dyn, reinterpret_cast<int *>(s_dyn + c.ncell + 1));
    }
  }
}

// ---------------------------------------------------------------- fused step

template <int TP, int METHOD, int PREC>
__global__ __launch_bounds__(1024) void k_step(SysConst c, SysPtrs p, int cur, int tail) {
  extern __shared__ unsigned s_tail_lds[];
  __shared__ SharedPairs sp;
  __shared__ BlockPartial s_waves[16];
  __shared__ int s_flag[2];
  __shared__ float s_cs2[kMaxPairs];
  const unsigned long long tstart = wall_clock64();
  stage_pairs(sp, c);
  // tail 2: a small system's list is built here, at the start of a step whose
  // rebuild flag is set (no list kernel in the chain): each wave builds the lists of
  // the block's own particles one after the other (the wave builder or the all-pairs
  // builder: the same lists as their list kernels), placing their sorted data; the
  // step then reads positions from the sorted copy, which the other workgroups may
  // not have placed yet
  const int build = tail == 2 ? p.ctl->rebuild : 0;
  // the friction of the step, read before the list build: the build's tallies are
  // atomics on the same control line from every workgroup, and a load queued behind
  // them waits several microseconds
  const double xi = c.thermostat ? p.ctl->xi : 0.0;
  if (build && threadIdx.x < kMaxPairs) s_cs2[threadIdx.x] = c.pt.cs2[threadIdx.x];
  __syncthreads();
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  // the positions of the step: the sorted copy on a build step after a sort, else in place
  const float4 *pos = p.pos[cur];
  if (build) {
    const int wv = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6), ppb = (int)blockDim.x / TP;
    const bool allp = c.list_kind == 4;  // all pairs: sorted only when a periodic re-sort was due
    const bool sorted = !allp || p.ctl->resorted != 0;
    if (sorted) pos = p.t_pos;
    int kept = 0, longest = 0;
    for (int q = wv; q < ppb; q += nw) {
      const int slot = lb * ppb + q;
      if (slot < c.n) {  // uniform across the wave
        int k;
        if (allp) {
          if (sorted && (threadIdx.x & 63) == 0) place_sorted(p, cur, slot, pos[slot]);
          k = list_allpairs_one(c, p, slot, s_cs2, pos, longest);
        } else {
          k = list_wave_one<true>(c, p, cur, slot, s_tail_lds + wv * kWaveCand, s_cs2, pos, p.cell_start, longest);
        }
        if ((threadIdx.x & 63) == 0) kept += k;
      }
    }
    list_tally(kept, longest, c.n_max, p.ctl);  // every thread of the block reaches this barrier once
    __syncthreads();  // the block's lists and placed data are visible to all its waves
  }
  const int gt = lb * blockDim.x + threadIdx.x;
  const int i = gt / TP, t = gt % TP;
  const bool active = i < c.n;
  float fx = 0.f, fy = 0.f, fz = 0.f, u = 0.f, w = 0.f;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  // integrator operands are loaded before the force loop so their latency overlaps it
  float4 vo = pi, l0 = pi, kc = pi;
  int4 im = make_int4(0, 0, 0, 0);
  double x64 = 0.0, y64 = 0.0, z64 = 0.0;
  if (active) {
    pi = pos[i];
    if (t == 0) {
      vo = p.vel[i];
      im = p.img[i];
      l0 = p.last[i];
      if (PREC == 1) kc = p.kahan[i];
      if (PREC == 2) {
        x64 = p.pos64[3 * i];
        y64 = p.pos64[3 * i + 1];
        z64 = p.pos64[3 * i + 2];
      }
    }
    force_lane<TP, METHOD, StepBatch<TP>::value, true>(i, t, pi, pos, (const int *)p.nbl, (const int *)p.nnb, sp, c, fx, fy,
                                             fz, u, w);
  }
  fx = lane_sum<TP>(fx);
  fy = lane_sum<TP>(fy);
  fz = lane_sum<TP>(fz);
  u = lane_sum<TP>(u);
  w = lane_sum<TP>(w);
  BlockPartial v = zero_partial();
  if (active && t == 0)
    integrate_one<PREC>(c, p, cur, i, pi, vo, im, l0, kc, x64, y64, z64, xi, fx, fy, fz, u, w, v,
                        tail && c.small_sort);
  v.t0 = tstart;
  v.t1 = wall_clock64();
  block_reduce(v, s_waves);
  if (threadIdx.x == 0) {
    store_to(&p.part[lb], v, tail != 0);
    // the list of this step has been consumed (with the tail, finish_step decides the flag)
    if (blockIdx.x == 0 && !tail) p.ctl->rebuild = 0;
  }
  // tail: the last workgroup to arrive ends the step (k_finish<0> not launched)
  if (tail && arrive_last(p.arrive, gridDim.x, blockIdx.x, &s_flag[0])) step_tail(c, p, gridDim.x, cur ^ 1, s_waves, s_flag, s_tail_lds);
}

// One workgroup after the step (MODE 0) or force-only (MODE 1) kernel: fixed-order
// float64 reduction of the G block partials (each thread sums its blocks in index
// order, then lanes by butterfly and waves in order), the Nose-Hoover update, the
// thermodynamic record, the displacement test that sets the rebuild flag, and for
// small systems the spatial sort for the next list build (positions pos[next]).
template <int MODE>
__global__ __launch_bounds__(1024) void k_finish(SysConst c, SysPtrs p, int G, int next) {
  __shared__ BlockPartial s_waves[16];
  __shared__ int s_rebuild, s_due;
  __shared__ unsigned s_cnt[MODE == 0 ? kSmallCells + 1 : 1];
  __shared__ int s_id[MODE == 0 ? kSmallN : 1];
  // the control words are final (the kernels before this one in the stream wrote
  // them), so they load beside the partials: one memory round trip instead of two
  CtlView cv{};
  if (MODE == 0 && threadIdx.x == 0) cv = load_ctl(p.ctl);
  BlockPartial a = zero_partial();
  for (int b = threadIdx.x; b < G; b += blockDim.x) {
    const BlockPartial q = p.part[b];
    a.pe += q.pe;
    a.w += q.w;
    a.ke_half += q.ke_half;
    a.ke_int += q.ke_int;
    a.disp2 = fmax(a.disp2, q.disp2);
    a.nonfinite |= q.nonfinite;
    a.t0 = q.t0 < a.t0 ? q.t0 : a.t0;
    a.t1 = q.t1 > a.t1 ? q.t1 : a.t1;
  }
  // threads at or past G hold zero partials: only the first (G + 63) / 64 waves are folded
  group_reduce(a, s_waves, (int)blockDim.x, (G + 63) / 64);
  if (threadIdx.x == 0) {
    Control *ctl = p.ctl;
    int rebuild = 0;
    if (MODE == 1) {
      Thermo *th = p.thermo;
      th->pe = a.pe;
      th->virial = a.w;
      th->ke = a.ke_half;  // kinetic energy of the stored (half-step) velocities
      th->ke_half = a.ke_half;
      th->temperature = 2.0 * a.ke_half / c.g;
      th->pressure = (2.0 * a.ke_half / 3.0 + a.w) / c.volume;
      th->xi = c.thermostat ? ctl->xi : 0.0;
      th->xi_integral = ctl->xi_int;
      th->h_conserved = a.ke_half + a.pe;
      th->max_nbrs = ctl->max_nbrs;
      th->n_rebuilds = ctl->n_rebuilds;
      th->step = ctl->step;
      if (a.nonfinite) ctl->error |= 1;
    } else {
      rebuild = finish_step(c, p, a, cv);
      s_due = resort_due(c, cv.n_rebuilds) ? 1 : 0;
    }
    s_rebuild = rebuild;
  }
  __syncthreads();
  if (MODE == 0 && s_rebuild && c.small_sort) {
    if (c.list_kind == 4 && !s_due) {
      if (threadIdx.x == 0) {
        begin_build(p.ctl);
        p.ctl->resorted = 0;
      }
    } else {
      sort_small_block<1024>(c, p, next, s_cnt, s_id);
    }
  }
}

// ---------------------------------------------------------------- persistent launches

// Butterfly of a BlockPartial over the 64 lanes of a wave (the first step of
// group_reduce), result valid in every lane.
__device__ __forceinline__ void wave_reduce(BlockPartial &v) {
  v.pe = wave_sum(v.pe);
  v.w = wave_sum(v.w);
  v.ke_half = wave_sum(v.ke_half);
  v.ke_int = wave_sum(v.ke_int);
  v.disp2 = wave_max(v.disp2);
  v.nonfinite = wave_or(v.nonfinite);
}

// a += q with the operations of the block and k_finish reductions.
__device__ __forceinline__ void fold(BlockPartial &a, const BlockPartial &q) {
  a.pe += q.pe;
  a.w += q.w;
  a.ke_half += q.ke_half;
  a.ke_int += q.ke_int;
  a.disp2 = fmax(a.disp2, q.disp2);
  a.nonfinite |= q.nonfinite;
}

// A pointer read from a descriptor in memory is generic to the compiler; loads
// through this global-address-space view compile to global (not flat) loads, which
// keep the list loads of the force loop pipelined.
#define SRMD_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ const SRMD_GLOBAL T *global_view(const T *q) {
  return (const SRMD_GLOBAL T *)q;
}

__device__ __forceinline__ float4 gload(const float4 *q, int i) {
  const raw_f4 v = ((const SRMD_GLOBAL raw_f4 *)q)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int4 gload(const int4 *q, int i) {
  const raw_i4 v = ((const SRMD_GLOBAL raw_i4 *)q)[i];
  return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int gload(const int *q, int i) { return ((const SRMD_GLOBAL int *)q)[i]; }

constexpr int kBatchThreads = 512;  // threads of a persistent workgroup
constexpr int kBatchWaves = kBatchThreads / 64;
constexpr int kCoopMaxGroups = 256;  // workgroups of one system (arrival words per parity)
constexpr int kMaxJobs = 64;         // jobs of one workgroup
constexpr int kLdsUnits = 64;        // wave partials of one piece kept in LDS (else in memory)

// Grid-wide barrier k (k = 1, 2, ... in one launch) of the G workgroups that share
// one system, over that system's array of arrival words (one per workgroup and
// barrier parity, cleared by the host before the launch).  Piece w publishes
// (k << 1) | bit in its word: an arrival costs one store and no read-modify-write on
// a shared counter, and bit carries a flag whose OR over the pieces every piece
// receives (the rebuild decision).  The first wave polls the G words of parity k & 1
// until each holds barrier k; two parities suffice because no piece can reach
// barrier k + 2 before every piece has left barrier k.  The wait is bounded (about
// one second of the 100 MHz device clock): on time-out the workgroup sets error bit 2
// and the kernel ends instead of hanging.  Release / acquire fences at agent scope
// order every store before the barrier against every load after it, once per
// workgroup: the release after each wave has waited for its own stores to complete
// (the L2 write-back acts on the whole cache), with the arrival store waiting for the
// write-back to complete; the acquire by the polling wave, whose invalidate of the
// compute unit's L1 and of the L2 precedes, through the workgroup barrier, every
// later load of the other waves.  With G = 1 the barrier is the workgroup barrier.
__device__ __forceinline__ bool coop_barrier(unsigned *flags, unsigned G, unsigned w, unsigned k, int bit,
                                             Control *ctl, int *s_ok, int *s_any) {
  if (G == 1) {
    __syncthreads();
    if (threadIdx.x == 0) *s_any = bit;
    __syncthreads();
    return true;
  }
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores have reached the L2
  __syncthreads();
  unsigned *slot = flags + (k & 1u) * kCoopMaxGroups;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // the L2 write-back must complete before the arrival is visible; the compiler's own
    // wait after the write-back is dropped when no store of this wave is outstanding
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(slot + w, (k << 1) | (unsigned)(bit != 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x < 64) {
    const unsigned long long t0 = wall_clock64();
    int ok = 1;
    bool any = false;
    while (true) {
      bool done = true, mine = false;
      for (unsigned l = threadIdx.x; l < G; l += 64) {
        const unsigned f = __hip_atomic_load(slot + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        done = done && (f >> 1) >= k;
        mine = mine || (f & 1u);
      }
      if (__all(done)) {
        any = __any(mine);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > 100000000ull) {
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) {
      if (!ok) atomicOr(&ctl->error, 4);
      *s_ok = ok;
      *s_any = any ? 1 : 0;
    }
  }
  __syncthreads();
  return *s_ok != 0;
}

// Positions of all n particles into LDS, eight loads in flight per thread.
__device__ __forceinline__ void fill_positions(float4 *dst, const float4 *src, int n) {
  for (int base = 0; base < n; base += 8 * kBatchThreads) {
    float4 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = gload(src, min(base + m * kBatchThreads + (int)threadIdx.x, n - 1));
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = base + m * kBatchThreads + (int)threadIdx.x;
      if (k < n) dst[k] = v[m];
    }
  }
}

// Small systems (N <= 8192, at most 8192 cells) advanced nsteps in one cooperative
// launch: one system over many workgroups (a single large enough system), many
// systems over the workgroups (a batch of replicas: the ensembles of small systems
// the paper's introduction points to), or both (a batch whose largest replicas are
// split over several workgroups and whose smallest share one).  Workgroup b runs the
// jobs jobs[job_off[b] .. job_off[b+1]) one after the other in every step.
//
// Piece w of g of a system owns the virtual blocks w, w + g, ... of that system's
// single-system step launch (G blocks of vb threads): its waves run the blocks' wave
// units (64 threads of that launch: the same particles, t_p lanes and list entries)
// with all positions of the step in LDS, and each block's wave partials are folded in
// index order into the block partial, as the step kernel does.  The partials buffer
// of a system holds two sets of G block partials (by step parity) and then one
// partial per wave unit.  After the barrier
// every piece reads the G block partials and repeats the fixed-order reduction of
// k_finish (so the thermostat needs no second barrier); piece 0 alone writes the
// record and the control block.  The rebuild decision travels with the barrier.  On
// a step that decides a rebuild, piece 0 sorts (as k_finish does), a barrier follows,
// the pieces build the lists of particles wave, wave + 8g, ..., and another barrier
// follows.  A system follows its single-system trajectory bit for bit at the same
// (tp, ppb), whatever the pieces and the other jobs of its workgroups.
//
// BIG: one larger system alone (more than 8192 particles or cells), positions read
// from device memory rather than LDS.  Its spatial sort is the four-phase counting
// sort of the launch chain, run by all pieces at the start of a step that rebuilds,
// with a grid barrier after each phase.
// Waves per SIMD the persistent kernel is compiled for: three from 16 lanes per
// particle up (measured +12 % at KA 4096, 32 bytes of spills), the register count's
// own two below, where three would spill 150 bytes per lane (the replica batch at
// t_p = 1 measured 1 % slower).
template <int TP>
struct kMultiWaves {
  static constexpr int value = TP >= 16 ? 3 : 1;
};

template <int TP, int METHOD, bool BIG>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(kMultiWaves<TP>::value))) void k_multi(const ReplicaDesc *__restrict__ reps,
                                                         const CoopJob *__restrict__ jobs,
                                                         const int *__restrict__ job_off, int nsteps,
                                                         int lds_bytes) {
  extern __shared__ float4 s_dyn[];
  __shared__ SharedPairs sp;
  __shared__ BlockPartial s_waves[16];
  __shared__ BlockPartial s_wp[kLdsUnits];
  __shared__ float s_cs2[kMaxPairs];
  __shared__ int s_ok, s_any, s_bit, s_due;
  __shared__ int s_rebuild[kMaxJobs], s_cur[kMaxJobs], s_resorted[kMaxJobs];
  __shared__ unsigned s_k[kMaxJobs];
  __shared__ double s_xi[kMaxJobs];
  __shared__ unsigned s_scan[16];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int j0 = job_off[blockIdx.x];
  const int nj = min(job_off[blockIdx.x + 1] - j0, kMaxJobs);
  // every piece reads its system's control block before piece 0 can write it
  for (int j = 0; j < nj; ++j) {
    const CoopJob J = jobs[j0 + j];
    const ReplicaDesc &R = reps[J.rep];
    if (tid == 0) {
      s_rebuild[j] = R.p.ctl->rebuild;
      s_resorted[j] = R.p.ctl->resorted;
      s_xi[j] = R.c.thermostat ? R.p.ctl->xi : 0.0;
      s_cur[j] = R.cur;
      s_k[j] = 1u;
    }
    if (!coop_barrier(R.p.bar_flags, J.g, J.w, 1u, 0, R.p.ctl, &s_ok, &s_any)) return;
  }
  bool prefilled = false;  // the positions of this step are already in LDS
  for (int step = 0; step < nsteps; ++step) {
    for (int j = 0; j < nj; ++j) {
      const CoopJob J = jobs[j0 + j];
      const ReplicaDesc &R = reps[J.rep];
      const SysConst &c = R.c;
      const SysPtrs &p = R.p;
      const int G = R.G, vb = R.vb, wpv = vb >> 6;
      const SRMD_GLOBAL int *nblg = global_view(p.nbl);
      const SRMD_GLOBAL int *nnbg = global_view(p.nnb);
      __syncthreads();  // the previous job's LDS use has ended
      int cur = s_cur[j];
      unsigned k = s_k[j];
      const int rebuild = s_rebuild[j];
      const double xi = s_xi[j];
      stage_pairs(sp, c);
      if (tid < kMaxPairs) s_cs2[tid] = c.pt.cs2[tid];
      if (tid == 0) s_bit = 0;
      __syncthreads();
      if (BIG && rebuild) {  // the counting sort of the launch chain, phase by phase
        const int base = J.w * kBatchThreads, stride = J.g * kBatchThreads;
        sort_bin(c, p, cur, base, stride);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
        if (J.w == 0 && tid == 0) begin_build(p.ctl);
        for (int b = J.w; b < scan_tiles(c.ncell); b += J.g) sort_scan_tile(c, p, b, s_scan);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
        sort_scatter(c, p, base + tid, stride, J.w == 0);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
        sort_gather(c, p, cur, base + tid, stride);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
      }
      if (!BIG && rebuild && c.list_kind == 4) {
        // all pairs from the positions of the step in LDS, no cells; after a periodic
        // re-sort from the sorted copy, with this piece's slots moved into place
        const bool resorted = s_resorted[j] != 0;
        fill_positions(s_dyn, resorted ? p.t_pos : p.pos[cur], c.n);
        if (resorted)
          for (int t = J.w * kBatchThreads + tid; t < c.n; t += J.g * kBatchThreads)
            place_sorted(p, cur, t, gload(p.t_pos, t));
        __syncthreads();
        int kept = 0, longest = 0;
        for (int t = J.w * kBatchWaves + wv; t < c.n; t += J.g * kBatchWaves) {
          const int kt = list_allpairs_one(c, p, t, s_cs2, s_dyn, longest);
          if (lane == 0) kept += kt;
        }
        list_tally(kept, longest, c.n_max, p.ctl);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
        prefilled = true;  // s_dyn holds this step's positions
      } else if (rebuild) {  // the spatial sort has been done (host request, end of step, or above)
        // the sorted positions and the cell starts go to LDS when they fit beside the
        // candidate windows, so the list build reads no device memory but its own list
        const int cs_words = (c.ncell + 1 + 3) & ~3;
        const bool in_lds = !BIG && 16 * c.n + 4 * cs_words + 4 * kBatchWaves * kWaveCand <= lds_bytes;
        const float4 *tpos = p.t_pos;
        const unsigned *cstart = p.cell_start;
        unsigned *cand = reinterpret_cast<unsigned *>(s_dyn) + wv * kWaveCand;
        if (in_lds) {
          fill_positions(s_dyn, p.t_pos, c.n);
          unsigned *s_cs = reinterpret_cast<unsigned *>(s_dyn + c.n);
          for (int q = tid; q <= c.ncell; q += kBatchThreads) s_cs[q] = gload((const int *)p.cell_start, q);
          __syncthreads();
          tpos = s_dyn;
          cstart = s_cs;
          cand = s_cs + cs_words + wv * kWaveCand;
        }
        // this piece's slots of the sorted arrays into place, coalesced (the list
        // build below only reads the sorted copies)
        for (int t = J.w * kBatchThreads + tid; t < c.n; t += J.g * kBatchThreads)
          place_sorted(p, cur, t, gload(p.t_pos, t));
        // one wave per cell (list_cell_particles), cells dealt round-robin over the
        // waves of all pieces, when each wave gets several cells; with about one cell
        // per wave the most crowded cell would set the pace, so then one wave per
        // particle.  The second half of the wave's window holds the counts.
        int kept = 0, longest = 0;
        const bool by_cell = 4 * J.g * kBatchWaves <= c.ncell;
        int *wcnt = reinterpret_cast<int *>(cand + kCellWindow);
        auto direct = [&](int i, int kk, int jj) {
          if (kk < c.n_max) p.nbl[nbl_addr(i, kk, c.tp, c.nvp)] = jj;
        };
        for (int t = J.w * kBatchWaves + wv; !by_cell && t < c.n; t += J.g * kBatchWaves) {
          const int kt = list_wave_one<false>(c, p, cur, t, cand, s_cs2, tpos, cstart, longest);
          if (lane == 0) kept += kt;
        }
        for (int cell = J.w * kBatchWaves + wv; by_cell && cell < c.ncell; cell += J.g * kBatchWaves) {
          const unsigned e1 = min(cstart[cell + 1], (unsigned)c.n), e0 = min(cstart[cell], e1);
          const int ne = (int)(e1 - e0);
          if (ne == 0) continue;  // uniform over the wave
          if (ne > kWaveCand - kCellWindow) {  // more particles than count slots: one at a time
            for (unsigned t = e0; t < e1; ++t) {
              const int kt = list_wave_one<false>(c, p, cur, (int)t, cand, s_cs2, tpos, cstart, longest);
              if (lane == 0) kept += kt;
            }
            continue;
          }
          for (int l = lane; l < ne; l += 64) wcnt[l] = 0;
          const int cx = cell % c.nc[0], cy = (cell / c.nc[0]) % c.nc[1], cz = cell / (c.nc[0] * c.nc[1]);
          list_cell_particles(c, p, cx, cy, cz, (int)e0, (int)e1, cand, wcnt, s_cs2, tpos, cstart, direct);
          for (int l = lane; l < ne; l += 64) {
            const int cn = wcnt[l];
            p.nnb[e0 + l] = min(cn, c.n_max);
            kept += min(cn, c.n_max);
            longest = max(longest, cn);
          }
        }
        list_tally(kept, longest, c.n_max, p.ctl);
        if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, 0, p.ctl, &s_ok, &s_any)) return;
      }
      if (!BIG && !prefilled) fill_positions(s_dyn, p.pos[cur], c.n);
      prefilled = false;
      __syncthreads();
      // positions of the step: the LDS copy, or device memory for a large system
      const float4 *spos = BIG ? (const float4 *)global_view(p.pos[cur]) : s_dyn;
      // this piece's wave units: unit q is wave q % wpv of owned block q / wpv; the
      // waves run their units without waiting for each other, and the wave partials
      // go to the system's partials buffer after the G block partials
      const int my_blocks = G > J.w ? (G - J.w + J.g - 1) / J.g : 0;
      const int my_units = my_blocks * wpv;
      // block partials alternate between two sets by step parity: a piece may write
      // the next step's partials while a slower piece still reads this step's
      BlockPartial *bpart = p.part + (step & 1) * G;
      // wave partials: in LDS (indexed by q) when this piece has few units, else in
      // the system's partials buffer (indexed by the unit)
      const bool wp_lds = my_units <= kLdsUnits;
      BlockPartial *wpart = p.part + 2 * G;
      for (int q = wv; q < my_units; q += kBatchWaves) {
        const int b = J.w + (q / wpv) * J.g;
        const int u = b * wpv + q % wpv;
        const int gt = u * 64 + lane;
        const int i = gt / TP, t = gt % TP;
        const bool active = i < c.n;
        float fx = 0.f, fy = 0.f, fz = 0.f, uu = 0.f, w = 0.f;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 vo = pi, l0 = pi, kc = pi;
        int4 im = make_int4(0, 0, 0, 0);
        if (active) {
          pi = BIG ? gload(p.pos[cur], i) : s_dyn[i];
          if (t == 0) {
            vo = gload(p.vel, i);
            im = gload(p.img, i);
            l0 = gload(p.last, i);
          }
          force_lane<TP, METHOD, Batch<TP>::value, true>(i, t, pi, spos, nblg, nnbg, sp, c, fx, fy, fz, uu, w);
        }
        fx = lane_sum<TP>(fx);
        fy = lane_sum<TP>(fy);
        fz = lane_sum<TP>(fz);
        uu = lane_sum<TP>(uu);
        w = lane_sum<TP>(w);
        BlockPartial v = zero_partial();
        if (active && t == 0)
          integrate_one<0>(c, p, cur, i, pi, vo, im, l0, kc, 0.0, 0.0, 0.0, xi, fx, fy, fz, uu, w, v);
        wave_reduce(v);
        if (lane == 0) {
          if (wp_lds)
            s_wp[q] = v;
          else
            wpart[u] = v;
          if (v.disp2 > c.half_skin2) s_bit = 1;
        }
      }
      __syncthreads();
      // owned block partials: each block's waves in index order (as group_reduce)
      for (int r = tid; r < my_blocks; r += kBatchThreads) {
        const int b = J.w + r * J.g;
        BlockPartial a = wp_lds ? s_wp[r * wpv] : wpart[b * wpv];
        for (int q = 1; q < wpv; ++q) fold(a, wp_lds ? s_wp[r * wpv + q] : wpart[b * wpv + q]);
        bpart[b] = a;
      }
      if (!coop_barrier(p.bar_flags, J.g, J.w, ++k, s_bit, p.ctl, &s_ok, &s_any)) return;
      // piece 0 loads the control words now, beside the partials of the reduction
      CtlView cv{};
      if (J.w == 0 && tid == 0) cv = load_ctl(p.ctl);
      // every piece: the reduction of k_finish (1024 threads, each thread here
      // standing in for threads tid and tid + 512 of that workgroup); with at most
      // 1024 blocks each thread's partials are loaded first, so that the positions
      // of the next step (loaded now when no rebuild is due and this is the
      // workgroup's only job) arrive in the same round trip
      BlockPartial a0 = zero_partial(), a1 = zero_partial();
      if (G <= 1024) {
        BlockPartial q0 = zero_partial(), q1 = zero_partial();
        if (tid < G) q0 = bpart[tid];
        if (tid + kBatchThreads < G) q1 = bpart[tid + kBatchThreads];
        prefilled = !BIG && nj == 1 && !s_any && step + 1 < nsteps;
        if (prefilled) fill_positions(s_dyn, p.pos[cur ^ 1], c.n);
        if (tid < G) fold(a0, q0);
        if (tid + kBatchThreads < G) fold(a1, q1);
      } else {
        for (int b = tid; b < G; b += 1024) fold(a0, bpart[b]);
        for (int b = tid + kBatchThreads; b < G; b += 1024) fold(a1, bpart[b]);
      }
      // a wave with no blocks holds zero partials, whose butterfly gives zeros again
      if (wv * 64 < G) wave_reduce(a0);
      if (kBatchThreads + wv * 64 < G) wave_reduce(a1);
      if (lane == 0) {
        s_waves[wv] = a0;
        s_waves[wv + kBatchWaves] = a1;
      }
      __syncthreads();
      if (tid == 0) {
        // the waves of k_finish that hold data (as its group_reduce folds them)
        BlockPartial a = s_waves[0];
        const int used = min(16, (G + 63) / 64);
        for (int q = 1; q < used; ++q) fold(a, s_waves[q]);
        a.t0 = 0ull;
        a.t1 = 0ull;
        if (J.w == 0) {
          finish_step(c, p, a, cv);  // the one writer of the control block
          s_due = resort_due(c, cv.n_rebuilds) ? 1 : 0;
        }
        if (c.thermostat) s_xi[j] = xi_next(c, xi, a.ke_half);
        s_rebuild[j] = s_any;  // = (max displacement^2 > (skin/2)^2), as finish_step decides
      }
      __syncthreads();
      cur ^= 1;
      if (!BIG && s_rebuild[j]) {
        // spatial sort of the new positions by piece 0, as k_finish does
        if (J.w == 0) {
          if (c.list_kind == 4 && !s_due) {  // all-pairs lists sort only when a re-sort is due
            if (tid == 0) {
              begin_build(p.ctl);
              p.ctl->resorted = 0;
            }
          } else {
            unsigned *scnt = reinterpret_cast<unsigned *>(s_dyn);
            sort_small_shared<1>(c, p, cur, scnt, reinterpret_cast<int *>(scnt + kSmallCells + 1));
          }
        }
        // every piece learns whether the build ahead starts from a re-sort (its
        // decision depends on the build count, which piece 0 holds)
        if (step + 1 < nsteps && !coop_barrier(p.bar_flags, J.g, J.w, ++k, J.w == 0 ? s_due : 0, p.ctl, &s_ok, &s_any))
          return;
        if (tid == 0) s_resorted[j] = c.list_kind == 4 ? s_any : 1;
      }
      if (tid == 0) {
        s_cur[j] = cur;
        s_k[j] = k;
      }
    }
  }
}

template <int TP, bool BIG>
static const void *multi_fn(int method) {
  return method == 0 ? (const void *)k_multi<TP, 0, BIG>
         : method == 1 ? (const void *)k_multi<TP, 1, BIG>
         : method == 2 ? (const void *)k_multi<TP, 2, BIG>
         : method == 3 ? (const void *)k_multi<TP, 3, BIG>
         : method == 4 ? (const void *)k_multi<TP, 4, BIG>
                       : (const void *)k_multi<TP, 5, BIG>;
}

// The persistent kernel for (tp, method); the large-system form exists for tp <= 8.
static const void *multi_fn_of(int tp, int method, bool big) {
  if (big) {
    switch (tp) {
      case 1: return multi_fn<1, true>(method);
      case 2: return multi_fn<2, true>(method);
      case 4: return multi_fn<4, true>(method);
      case 8: return multi_fn<8, true>(method);
      default: return nullptr;
    }
  }
  switch (tp) {
    case 1: return multi_fn<1, false>(method);
    case 2: return multi_fn<2, false>(method);
    case 4: return multi_fn<4, false>(method);
    case 8: return multi_fn<8, false>(method);
    case 16: return multi_fn<16, false>(method);
    case 32: return multi_fn<32, false>(method);
    case 64: return multi_fn<64, false>(method);
    default: return nullptr;
  }
}

bool multi_big_supported(int tp) { return multi_fn_of(tp, 0, true) != nullptr; }

// Launch k_multi over nwg workgroups.  cooperative: some system is split over
// several workgroups, which must then all be resident at once.
hipError_t launch_multi(int tp, int method, bool big, int nwg, size_t lds, hipStream_t st, const ReplicaDesc *reps,
                        const CoopJob *jobs, const int *job_off, int nsteps, bool cooperative) {
  const void *fn = multi_fn_of(tp, method, big);
  if (!fn || nwg < 1) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int lds_bytes = (int)lds;
  void *args[] = {&reps, &jobs, &job_off, &nsteps, &lds_bytes};
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(kBatchThreads), args, (unsigned)lds, st);
  return hipLaunchKernel(fn, dim3(nwg), dim3(kBatchThreads), args, lds, st);
}

// Workgroups of the persistent kernel the device holds at once (at most 256).
int multi_max_groups(int tp, int method, bool big, size_t lds) {
  const void *fn = multi_fn_of(tp, method, big);
  if (!fn) return 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchThreads, lds) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return std::min(per_cu * cus, kCoopMaxGroups);
}

int multi_max_jobs() { return kMaxJobs; }

// Dynamic LDS of the persistent kernel: the positions of a step, the sort's scratch,
// and where it fits in 150 KiB, the list build's copies of the sorted positions and
// the cell starts beside the candidate windows (up to 4096 cells counted).
size_t batch_lds_bytes(int n_max_particles) {
  const size_t pos = 16 * (size_t)n_max_particles;
  const size_t scratch = 4 * (size_t)(kSmallCells + 1 + kSmallN);
  const size_t cand = 4 * (size_t)(kBatchWaves * kWaveCand);
  const size_t listing = pos + 4 * (size_t)(4096 + 4) + cand;
  size_t b = std::max(pos, std::max(scratch, cand));
  if (listing <= 150 * 1024) b = std::max(b, listing);
  return b;
}

int batch_max_particles() { return kSmallN; }

// Dynamic LDS of the large-system persistent kernel: the list build's candidate windows.
size_t big_lds_bytes() { return 4 * (size_t)(kBatchWaves * kWaveCand); }

// ---------------------------------------------------------------- start of a stepping call

// One launch at the start of srmd_step: the call's trace settings go into the
// control block, and the dynamic state the call starts from (positions, velocities,
// last-build positions, images and ids, precision residuals and the control block
// itself) is copied into the replay snapshot.
__global__ __launch_bounds__(256) void k_call_begin(SysConst c, SysPtrs p, Snapshot snap, int cur, int thermo_every,
                                                    long long trace_cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    Control k = *p.ctl;
    k.thermo_every = thermo_every;
    k.trace_cap = trace_cap;
    k.n_records = 0;
    *p.ctl = k;
    *snap.ctl = k;
  }
  if (i < c.n) {
    snap.pos[i] = p.pos[cur][i];
    snap.vel[i] = p.vel[i];
    snap.last[i] = p.last[i];
    snap.img[i] = p.img[i];
    if (snap.kahan) snap.kahan[i] = p.kahan[i];
    if (snap.pos64) {
      snap.pos64[3 * i] = p.pos64[3 * i];
      snap.pos64[3 * i + 1] = p.pos64[3 * i + 1];
      snap.pos64[3 * i + 2] = p.pos64[3 * i + 2];
    }
  }
}

// ---------------------------------------------------------------- stateless force evaluation

// Set-up of a stateless force evaluation in caller-provided scratch: the control
// block cleared with a rebuild requested, and the caller's positions (x, y, z per
// particle, wrapped into [-L/2, L/2) as srmd_create wraps them) and types stored in
// original order with zero velocities, zero images and identity ids; *status
// cleared.  A type out of range is stored as 0 with its image x counter set to 1
// (reported by k_direct_out), so that no table lookup leaves the pair tables.
__global__ __launch_bounds__(256) void k_direct_init(SysConst c, SysPtrs p, const float *__restrict__ xyz,
                                                     const int *__restrict__ type, int *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    Control k;
    int *w = reinterpret_cast<int *>(&k);
    for (int q = 0; q < (int)(sizeof(Control) / sizeof(int)); ++q) w[q] = 0;
    k.rebuild = 1;
    *p.ctl = k;
    *status = 0;
  }
  if (i >= c.n) return;
  float r[3];
  for (int d = 0; d < 3; ++d) {
    const double x = (double)xyz[3 * i + d], L = c.Ld[d];
    float f = (float)(x - L * floor(x / L + 0.5));
    if (f >= c.halfL[d]) f -= c.L[d];
    if (f < -c.halfL[d]) f += c.L[d];
    r[d] = f;
  }
  int ty = type[i];
  const int bad = (ty < 0 || ty >= c.ntypes) ? 1 : 0;
  if (bad) ty = 0;
  p.pos[0][i] = make_float4(r[0], r[1], r[2], __int_as_float(ty));
  p.vel[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  p.img[i] = make_int4(bad, 0, 0, i);
}

// End of a stateless force evaluation: forces in original particle order, the
// float64 potential energy and virial, and into *status the control block's error
// bits (bit 0 non-finite force, bit 1 list capacity exceeded) and bit 2 for a type
// out of range.
__global__ __launch_bounds__(256) void k_direct_out(SysConst c, SysPtrs p, float *__restrict__ force,
                                                    double *__restrict__ energy, int *status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    energy[0] = p.thermo->pe;
    energy[1] = p.thermo->virial;
    const int e = p.ctl->error & 3;
    if (e) atomicOr(status, e);
  }
  if (t >= c.n) return;
  const int4 im = p.img[t];
  if (im.x != 0) atomicOr(status, 4);
  const int id = im.w;
  if (id < 0 || id >= c.n) return;
  const float4 f = p.force[t];
  force[3 * id] = f.x;
  force[3 * id + 1] = f.y;
  force[3 * id + 2] = f.z;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_direct_init(hipStream_t st, const SysConst &c, const SysPtrs &p, const float *xyz, const int *type,
                              int *status) {
  hipLaunchKernelGGL(k_direct_init, dim3((c.n + 255) / 256), dim3(256), 0, st, c, p, xyz, type, status);
  return hipGetLastError();
}

hipError_t launch_direct_out(hipStream_t st, const SysConst &c, const SysPtrs &p, float *force, double *energy,
                             int *status) {
  hipLaunchKernelGGL(k_direct_out, dim3((c.n + 255) / 256), dim3(256), 0, st, c, p, force, energy, status);
  return hipGetLastError();
}

hipError_t launch_call_begin(hipStream_t st, const SysConst &c, const SysPtrs &p, const Snapshot &snap, int cur,
                             int thermo_every, long long trace_cap) {
  hipLaunchKernelGGL(k_call_begin, dim3((c.n + 255) / 256), dim3(256), 0, st, c, p, snap, cur, thermo_every, trace_cap);
  return hipGetLastError();
}

template <int TP>
static hipError_t launch_step_tp(int method, int prec, dim3 g, dim3 b, hipStream_t st, const SysConst &c,
                                 const SysPtrs &p, int cur, int tail, size_t lds) {
#define SRMD_STEP_CASE(M, P)                                                   \
  if (method == M && prec == P) {                                              \
    hipLaunchKernelGGL((k_step<TP, M, P>), g, b, lds, st, c, p, cur, tail);    \
    return hipGetLastError();                                                  \
  }
  SRMD_STEP_CASE(0, 0) SRMD_STEP_CASE(0, 1) SRMD_STEP_CASE(0, 2)
  SRMD_STEP_CASE(1, 0) SRMD_STEP_CASE(1, 1) SRMD_STEP_CASE(1, 2)
  SRMD_STEP_CASE(2, 0) SRMD_STEP_CASE(2, 1) SRMD_STEP_CASE(2, 2)
  SRMD_STEP_CASE(3, 0) SRMD_STEP_CASE(3, 1) SRMD_STEP_CASE(3, 2)
  SRMD_STEP_CASE(4, 0) SRMD_STEP_CASE(4, 1) SRMD_STEP_CASE(4, 2)
  SRMD_STEP_CASE(5, 0) SRMD_STEP_CASE(5, 1) SRMD_STEP_CASE(5, 2)
#undef SRMD_STEP_CASE
  return hipErrorInvalidValue;
}

template <int TP>
static hipError_t launch_force_tp(int method, dim3 g, dim3 b, hipStream_t st, const SysConst &c, const SysPtrs &p,
                                  int cur) {
  if (method == 0) hipLaunchKernelGGL((k_force<TP, 0>), g, b, 0, st, c, p, cur);
  else if (method == 1) hipLaunchKernelGGL((k_force<TP, 1>), g, b, 0, st, c, p, cur);
  else if (method == 2) hipLaunchKernelGGL((k_force<TP, 2>), g, b, 0, st, c, p, cur);
  else if (method == 3) hipLaunchKernelGGL((k_force<TP, 3>), g, b, 0, st, c, p, cur);
  else if (method == 4) hipLaunchKernelGGL((k_force<TP, 4>), g, b, 0, st, c, p, cur);
  else if (method == 5) hipLaunchKernelGGL((k_force<TP, 5>), g, b, 0, st, c, p, cur);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// tail = 1: the step kernel ends the step in its last workgroup (no k_finish<0>
// launch); lds = tail_lds_bytes for small systems, else 0.
hipError_t launch_step(int tp, int method, int prec, int blocks, int threads, hipStream_t st, const SysConst &c,
                       const SysPtrs &p, int cur, int tail, size_t lds) {
  const dim3 g(blocks), b(threads);
  switch (tp) {
    case 1: return launch_step_tp<1>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 2: return launch_step_tp<2>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 4: return launch_step_tp<4>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 8: return launch_step_tp<8>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 16: return launch_step_tp<16>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 32: return launch_step_tp<32>(method, prec, g, b, st, c, p, cur, tail, lds);
    case 64: return launch_step_tp<64>(method, prec, g, b, st, c, p, cur, tail, lds);
    default: return hipErrorInvalidValue;
  }
}

// Dynamic LDS of a step kernel with the tail: the spatial sort's arrays for small
// systems (sorted in the tail), none otherwise; with the list built in the step
// (tail 2), at least the wave builder's candidate windows (the two uses alias).
size_t tail_lds_bytes(const SysConst &c, int threads, int tail) {
  const size_t sort = c.small_sort ? tail_sort_lds(c.n, c.ncell) : 0;
  const size_t windows = tail == 2 && c.list_kind == 1 ? sizeof(unsigned) * kWaveCand * (size_t)(threads / 64) : 0;
  return std::max(sort, windows);
}

// Bytes of a system's arrival counters (zeroed at allocation).
size_t arrive_bytes() { return kArriveBytes; }

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

hipError_t launch_finish(int mode, int G, int next, hipStream_t st, const SysConst &c, const SysPtrs &p) {
  if (mode == 0) hipLaunchKernelGGL((k_finish<0>), dim3(1), dim3(1024), 0, st, c, p, G, next);
  else hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(1024), 0, st, c, p, G, next);
  return hipGetLastError();
}

// Sort requested by the host for a small system (the multi-kernel sort of large
// systems always runs at the start of the step, gated on the flag).
hipError_t launch_host_sort(hipStream_t st, const SysConst &c, const SysPtrs &p, int cur) {
  if (!c.small_sort) return hipSuccess;
  hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(1024), 0, st, c, p, cur);
  return hipGetLastError();
}

// Start-of-step rebuild chain: list build (small systems; the sort ran earlier) or
// the multi-kernel sort followed by the list build (large systems).
hipError_t launch_rebuild(hipStream_t st, const SysConst &c, const SysPtrs &p, int cur) {
  const int tb = 256;
  const int gb = c.list_blocks;
  if (!c.small_sort) {
    hipLaunchKernelGGL(k_bin, dim3(gb), dim3(tb), 0, st, c, p, cur);
    hipLaunchKernelGGL(k_scan, dim3(scan_tiles(c.ncell)), dim3(256), 0, st, c, p);
    hipLaunchKernelGGL(k_scatter, dim3(gb), dim3(tb), 0, st, c, p);
    hipLaunchKernelGGL(k_gather, dim3(gb), dim3(tb), 0, st, c, p, cur);
  }
  if (c.list_kind == 4) {
    const int lb = (c.n + 3) / 4;
    hipLaunchKernelGGL(k_list_allpairs, dim3(lb), dim3(tb), 0, st, c, p, cur);
  } else if (c.list_kind == 1) {
    const int lb = (c.n + 3) / 4;
    hipLaunchKernelGGL(k_list_wave, dim3(lb), dim3(tb), 0, st, c, p, cur);
  } else if (c.list_kind == 2) {
    hipLaunchKernelGGL(k_list_thread, dim3(gb), dim3(tb), 0, st, c, p, cur);
  } else if (c.list_kind == 5) {
    hipLaunchKernelGGL(k_list_row, dim3(c.nc[1] * c.nc[2]), dim3(256), 0, st, c, p, cur);
  } else {
    const int lb = (c.n + kCellSlots - 1) / kCellSlots;
    hipLaunchKernelGGL(k_list_cell, dim3(lb), dim3(128), 0, st, c, p, cur);
  }
  return hipGetLastError();
}

}  // namespace srmd
