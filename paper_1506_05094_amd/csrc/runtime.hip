// Host runtime and C-ABI of libsrmd: device state, parameter tables, the cell
// grid and list capacity, the graph-captured step chunks, list-overflow recovery
// and the original-order views of the state.
#include <algorithm>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/srmd.h"
#include "srmd_internal.h"

namespace srmd {
hipError_t launch_step(int tp, int method, int prec, int blocks, int threads, hipStream_t st, const SysConst &c,
                       const SysPtrs &p, int cur, int tail, size_t lds);
size_t tail_lds_bytes(const SysConst &c, int threads, int tail);
size_t arrive_bytes();
hipError_t launch_force(int tp, int method, int blocks, int threads, hipStream_t st, const SysConst &c,
                        const SysPtrs &p, int cur);
hipError_t launch_rebuild(hipStream_t st, const SysConst &c, const SysPtrs &p, int cur);
hipError_t launch_finish(int mode, int G, int next, hipStream_t st, const SysConst &c, const SysPtrs &p);
hipError_t launch_host_sort(hipStream_t st, const SysConst &c, const SysPtrs &p, int cur);
hipError_t launch_call_begin(hipStream_t st, const SysConst &c, const SysPtrs &p, const Snapshot &snap, int cur,
                             int thermo_every, long long trace_cap);
hipError_t launch_direct_init(hipStream_t st, const SysConst &c, const SysPtrs &p, const float *xyz, const int *type,
                              int *status);
hipError_t launch_direct_out(hipStream_t st, const SysConst &c, const SysPtrs &p, float *force, double *energy,
                             int *status);
bool small_sort_fits(int n, int ncell);
size_t batch_lds_bytes(int n_max_particles);
int batch_max_particles();
hipError_t launch_multi(int tp, int method, bool big, int nwg, size_t lds, hipStream_t st, const ReplicaDesc *reps,
                        const CoopJob *jobs, const int *job_off, int nsteps, bool cooperative);
int multi_max_groups(int tp, int method, bool big, size_t lds);
bool multi_big_supported(int tp);
size_t big_lds_bytes();
int multi_max_jobs();
}  // namespace srmd

using namespace srmd;

namespace {

thread_local std::string g_thread_error;

struct Allocator {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  void *ctx = nullptr;
};
Allocator g_alloc;  // process-wide hook

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  Allocator how;
};

constexpr int kChunk = 64;  // steps per captured graph (even: the position buffers alternate)
constexpr size_t kTailLdsMax = 60 * 1024;  // dynamic LDS of a step kernel that sorts in its last workgroup
constexpr int kTailAutoBlocks = 256;       // largest small-system grid that ends its steps itself by default
constexpr int kBuildPerWave = 8;          // most particles a wave of the step kernel builds the lists of
constexpr int kBuildPerWaveAllPairs = 2;  // the same with all-pairs lists (N candidates each: measured slower at 4 and 8)
constexpr double kTunerListKeep = 1.05;   // list methods within 5 % of the fastest at the default layout go on to phase II
constexpr int kPersistChunk = 500;  // steps per launch of the persistent kernel (even)

}  // namespace

struct srmd_system {
  int n = 0, ntypes = 0;
  srmd_precision prec = SRMD_PREC_F32;
  float Lf[3] = {0, 0, 0};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double mass[kMaxTypes] = {1, 1, 1, 1};
  // potential
  double sigma[kMaxPairs] = {}, eps[kMaxPairs] = {}, rc[kMaxPairs] = {};
  bool pair_given[kMaxPairs] = {};
  int method = -1;
  int pot = -1;                         // 0 Lennard-Jones, 1 two-power (srmd_set_pair_mie), 2..6 the further
                                        // potentials (srmd_set_pair_potential); -1 none yet
  double mie_a[kMaxPairs] = {}, mie_b[kMaxPairs] = {};
  int mie_m[kMaxPairs] = {}, mie_n[kMaxPairs] = {};
  double gen_p[kMaxPairs][4] = {};      // parameters of a further potential
  bool coulomb = false;                 // shifted-force Coulomb term on (srmd_set_coulomb_sf)
  double charge[kMaxTypes] = {0, 0, 0, 0};
  double rcc = 0.0;                     // its cutoff
  double skin = 0.3;
  // integrator
  bool integrator_set = false;
  int thermostat = 0;
  double dt = 0.0, T0 = 0.0, tau = 0.0;
  // launch shape
  int tp_req = 0, ppb_req = 0, tp = 0, ppb = 0;
  int tp_tuned = 0, ppb_tuned = 0;
  int sort_mode = 0, list_mode = 0;  // 0 auto; sort 1 one workgroup / 2 multi-kernel; list 1 wave / 2 thread / 3 cell / 4 all pairs
  int sort_every = 0;                // all-pairs lists: spatial sort at every k-th build (0: never)
  int tail_req = -1;                 // launch chains: step kernel ends the step (1), also builds small systems' lists (2), k_finish (0), automatic (-1)
  bool sort_pending = false;         // a host-requested rebuild still needs its one-workgroup sort
  int persist_req = 0;               // persistent kernel: 0 off, -1 automatic group count, > 0 groups
  bool persist_set = false;          // persist_req given by the caller (else the tuned choice applies)
  int persist_tuned = 0;             // choice of srmd_autotune
  int persist_groups = 0;            // resolved workgroup count, 0 = launch chains
  std::string persist_err;           // why the requested persistent mode cannot run
  ReplicaDesc *d_desc = nullptr;     // persistent launch tables (one system, persist_groups jobs)
  CoopJob *d_jobs = nullptr;
  int *d_job_off = nullptr;
  int jobs_cap = 0, jobs_g = 0;      // capacity and current size of the job table
  ReplicaDesc host_desc{};           // last uploaded descriptor
  bool desc_valid = false;
  // derived layout
  bool dirty = true;  // SysConst must be rebuilt
  SysConst c{};
  SysPtrs p{};
  int cur = 0;
  int n_max = 0, nvp = 0, ncell_alloc = 0;
  long long nbl_alloc = 0;
  long long trace_alloc = 0;
  int part_alloc = 0;
  std::vector<DevBuf> bufs;
  // snapshot for list-overflow replay
  Snapshot snap{};
  Control *h_ctl = nullptr;  // pinned host copy of the control block, read back once per call
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::string err;
};

namespace {

srmd_status fail(srmd_system *s, srmd_status st, const std::string &msg) {
  if (s)
    s->err = msg;
  else
    g_thread_error = msg;
  return st;
}

#define HIPCHK(s, call)                                                                               \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return fail((s), SRMD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));                 \
  } while (0)

// One device buffer from the allocator hook in force (hipMalloc without one); the
// buffer remembers how it was made so that it is released the same way.
DevBuf raw_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  DevBuf b;
  b.bytes = bytes;
  b.how = g_alloc;
  if (g_alloc.alloc) {
    b.ptr = g_alloc.alloc(bytes, g_alloc.ctx);
  } else {
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) b.ptr = nullptr;
  }
  return b;
}

void raw_free(DevBuf &b) {
  if (b.ptr) {
    if (b.how.free_fn)
      b.how.free_fn(b.ptr, b.how.ctx);
    else if (!b.how.alloc)
      (void)hipFree(b.ptr);
  }
  b = DevBuf{};
}

void *dev_alloc(srmd_system *s, size_t bytes) {
  DevBuf b = raw_alloc(bytes);
  if (!b.ptr) return nullptr;
  s->bufs.push_back(b);
  return b.ptr;
}

void dev_free(srmd_system *s, void *ptr) {
  if (!ptr) return;
  for (size_t k = 0; k < s->bufs.size(); ++k) {
    if (s->bufs[k].ptr == ptr) {
      raw_free(s->bufs[k]);
      s->bufs.erase(s->bufs.begin() + (long)k);
      return;
    }
  }
}

void drop_graphs(srmd_system *s) {
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
}

int pair_index(const srmd_system *s, int a, int b) { return a * s->ntypes + b; }

double lj_u(double r, double sig, double eps) {
  const double sr = sig / r;
  const double sr6 = sr * sr * sr * sr * sr * sr;
  return 4.0 * eps * (sr6 * sr6 - sr6);
}

// A s^m - B s^n with s = sig / r, and its force -dU/dr
double mie_u(double r, double A, double B, int m, int n, double sig) {
  const double s = sig / r;
  return A * std::pow(s, m) - B * std::pow(s, n);
}

double mie_f(double r, double A, double B, int m, int n, double sig) {
  const double s = sig / r;
  return (m * A * std::pow(s, m) - n * B * std::pow(s, n)) / r;
}

double lj_f(double r, double sig, double eps) {
  const double sr = sig / r;
  const double sr6 = sr * sr * sr * sr * sr * sr;
  return 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r;
}

// Energy and force -dU/dr of a further potential (kinds 2..6, srmd_set_pair_potential)
// in float64, for its values at the cutoff.
void further_uf(int kind, const double *p, double sig, double r, double *u, double *f) {
  if (kind == 2) {  // Yukawa
    const double e = std::exp(-p[1] * (r - sig));
    *u = p[0] * sig / r * e;
    *f = *u * (1.0 + p[1] * r) / r;
  } else if (kind == 3) {  // Buckingham
    const double e = p[0] * std::exp(-r / p[1]), d6 = p[2] / std::pow(r, 6);
    *u = e - d6;
    *f = e / p[1] - 6.0 * d6 / r;
  } else if (kind == 4) {  // Gaussian core
    const double e = p[0] * std::exp(-(r / sig) * (r / sig));
    *u = e;
    *f = 2.0 * r / (sig * sig) * e;
  } else if (kind == 5) {  // Dzugutov
    const double x = r / sig;
    double uu = 0.0, du = 0.0;
    if (x < 1.87) {
      const double q = 1.0 / (x - 1.87), e = std::exp(1.1 * q), xm = std::pow(x, -16.0);
      uu += 5.82 * (xm - 1.28) * e;
      du += 5.82 * e * (-16.0 * xm / x - (xm - 1.28) * 1.1 * q * q);
    }
    if (x < 1.94) {
      const double q = 1.0 / (x - 1.94), e = 1.28 * std::exp(0.27 * q);
      uu += e;
      du -= e * 0.27 * q * q;
    }
    *u = p[0] * uu;
    *f = -p[0] * du / sig;
  } else {  // Girifalco
    const double x = r / sig, a = x - 1.0, b = x + 1.0;
    auto br = [&](int k, double *v, double *dv) {
      const double ak = std::pow(a, k), bk = std::pow(b, k), xk = std::pow(x, k + 1);
      *v = 1.0 / (x * ak) + 1.0 / (x * bk) - 2.0 / xk;
      *dv = -1.0 / (x * x * ak) - k / (x * ak * a) - 1.0 / (x * x * bk) - k / (x * bk * b) + 2.0 * (k + 1) / (xk * x);
    };
    double at, dat, rp, drp;
    br(3, &at, &dat);
    br(9, &rp, &drp);
    *u = -p[0] * at + p[1] * rp;
    *f = (p[0] * dat - p[1] * drp) / sig;
  }
}

double rc_max(const srmd_system *s) {
  double m = s->coulomb ? s->rcc : 0.0;
  for (int a = 0; a < s->ntypes * s->ntypes; ++a)
    if (s->pair_given[a]) m = std::max(m, s->rc[a]);
  return m;
}

// The method index the kernels are instantiated for: the Lennard-Jones cutoff
// method, 3 for shifted-force Lennard-Jones plus shifted-force Coulomb, 4 for the
// two-power potential (any cutoff method).
int kmethod(const srmd_system *s) { return s->coulomb ? 3 : s->pot == 1 ? 4 : s->pot >= 2 ? 5 : s->method; }

bool all_pairs_given(const srmd_system *s) {
  for (int a = 0; a < s->ntypes * s->ntypes; ++a)
    if (!s->pair_given[a]) return false;
  return true;
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Default threads per particle: enough lanes in flight for the chip (about 32k, or
// 64k for the persistent kernel, which then spreads over more compute units), the
// MI355X version of the paper's rule that N * t_p should exceed the core count
// several times over (section 8, autotuner choices).
void launch_of(const srmd_system *s, int *tp_out, int *ppb_out) {
  int tp = s->tp_req, ppb = s->ppb_req;
  if (tp == 0) {
    if (s->tp_tuned) {
      tp = s->tp_tuned;
      ppb = s->ppb_tuned;
    } else {
      // enough lanes to fill the device, and for long lists (the Coulomb term's
      // several hundred entries) at most about 64 entries per lane; the expected
      // length is the mean count inside r_c,max + s
      const bool persistent = s->persist_set ? s->persist_req != 0 : s->persist_tuned != 0;
      const int lanes = persistent ? 65536 : 32768;
      const double reach = rc_max(s) + s->skin;
      const double V = (double)s->Lf[0] * (double)s->Lf[1] * (double)s->Lf[2];
      const double expected = 4.0 / 3.0 * M_PI * reach * reach * reach * (double)s->n / V;
      const int by_list = (int)std::min(64.0, expected / 64.0);
      tp = std::min(32, pow2_at_least(std::max(1, std::max(lanes / std::max(1, s->n), by_list))));
      ppb = 0;
    }
  }
  if (ppb == 0) ppb = std::max(1, 256 / tp);
  *tp_out = tp;
  *ppb_out = ppb;
}

void resolve_launch(srmd_system *s) { launch_of(s, &s->tp, &s->ppb); }

srmd_status h2d_sync(srmd_system *s, void *dst, const void *src, size_t bytes) {
  HIPCHK(s, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

srmd_status set_ctl_int(srmd_system *s, size_t offset, int value) {
  return h2d_sync(s, reinterpret_cast<char *>(s->p.ctl) + offset, &value, sizeof(int));
}

srmd_status request_rebuild(srmd_system *s) {
  s->sort_pending = true;
  return set_ctl_int(s, offsetof(Control, rebuild), 1);
}

// A host-requested rebuild of a small system needs its sort before the list build.
srmd_status flush_host_sort(srmd_system *s) {
  if (!s->sort_pending) return SRMD_OK;
  s->sort_pending = false;
  HIPCHK(s, launch_host_sort(s->stream, s->c, s->p, s->cur));
  return SRMD_OK;
}

int step_blocks(const srmd_system *s) { return (int)(((long long)s->n * s->tp + s->tp * s->ppb - 1) / (s->tp * s->ppb)); }

// Dynamic LDS of the persistent kernel for this system.
size_t persist_lds(const srmd_system *s) { return s->c.small_sort ? batch_lds_bytes(s->n) : big_lds_bytes(); }

// Workgroups of the persistent kernel (0: launch chains): by default one workgroup
// of 512 threads per 8 waves of the step launch, so each wave takes one wave of it.
void resolve_persistent(srmd_system *s) {
  s->persist_groups = 0;
  s->persist_err.clear();
  const int preq = s->persist_set ? s->persist_req : s->persist_tuned;
  if (preq == 0) return;
  if (s->prec != SRMD_PREC_F32) {
    s->persist_err = "the persistent kernel needs float32 positions";
    return;
  }
  if (!s->c.small_sort && !multi_big_supported(s->tp)) {
    s->persist_err = "the persistent kernel takes a system of more than 8192 particles or cells with tp <= 8 only";
    return;
  }
  const int threads = s->tp * s->ppb;
  const int units = step_blocks(s) * (threads / 64);
  const int cap = multi_max_groups(s->tp, kmethod(s), !s->c.small_sort, persist_lds(s));
  int want = preq > 0 ? preq : std::max(1, (units + 7) / 8);
  if (preq < 0) want = std::min(want, cap);
  if (want > cap || want < 1)
    s->persist_err = "the persistent kernel's workgroups do not all fit on the device at once";
  else
    s->persist_groups = want;
}

// The kernel constants of s: launch shape, cell grid, list capacity and the
// per-type-pair tables (host only; no device memory is touched).
srmd_status fill_const(srmd_system *s) {
  resolve_launch(s);
  SysConst &c = s->c;
  std::memset(&c, 0, sizeof(c));
  c.n = s->n;
  c.ntypes = s->ntypes;
  const double rcm = rc_max(s);
  const double reach = rcm + s->skin;
  double V = 1.0;
  for (int k = 0; k < 3; ++k) {
    c.L[k] = s->Lf[k];
    c.invL[k] = (float)(1.0 / (double)s->Lf[k]);
    c.halfL[k] = 0.5f * s->Lf[k];
    c.Ld[k] = (double)s->Lf[k];
    V *= c.Ld[k];
    if (!(reach < 0.5 * c.Ld[k]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
    // cells of side at least (r_c + s)/2 (paper section 7), with a relative margin
    // of 1e-5 so that float32 rounding of the cell coordinate never moves a listed
    // neighbour outside the +-2 stencil
    const double cmin = 0.5 * reach * (1.0 + 1e-5);
    int nc = (int)std::floor(c.Ld[k] / cmin);
    nc = std::max(1, std::min(nc, 1 << 10));
    c.nc[k] = nc;
    c.cscale[k] = (float)((double)nc / c.Ld[k]);
    if (nc < 5) c.full_axis |= 1 << k;
  }
  c.ncell = c.nc[0] * c.nc[1] * c.nc[2];
  c.volume = V;
  const bool fits = small_sort_fits(s->n, c.ncell);
  c.small_sort = (s->sort_mode == 0 || s->sort_mode == 1) && fits ? 1 : 0;
  // measured on MI355X (LJ fluid): the cell builder is fastest from 16k to 64k particles and
  // the thread builder from 256k on; the autotuner compares all three
  c.list_kind = s->list_mode != 0 ? s->list_mode : s->n <= 4096 ? 1 : s->n <= 131072 ? 3 : 2;
  if (c.list_kind == 4 && !c.small_sort)
    return fail(s, SRMD_EINVAL, "the all-pairs list build takes systems of at most 8192 particles and 8192 cells "
                                "with the one-workgroup sort mode");
  c.list_blocks = std::max(1, std::min((s->n + 255) / 256, 2048));
  c.pot_kind = s->pot >= 2 ? s->pot : 0;
  c.sort_every = c.list_kind == 4 ? s->sort_every : 0;
  // list capacity: 1.5 x the mean count in a sphere of radius r_c + s, + 32 (rounded to 32)
  const double rho = s->n / V;
  int nmax = (int)std::ceil(1.5 * 4.0 / 3.0 * M_PI * reach * reach * reach * rho + 32.0);
  nmax = (nmax + 63) / 64 * 64;     // a multiple of every tp, so the list layout tiles exactly
  nmax = std::max(nmax, s->n_max);  // never shrink after an overflow regrow
  nmax = std::min(nmax, (s->n + 63) / 64 * 64);
  s->n_max = nmax;
  c.n_max = nmax;
  c.nvp = (s->n + 63) / 64 * 64;
  c.tp = s->tp;
  c.dt = (float)s->dt;
  c.dtd = s->dt;
  c.T0 = s->T0;
  c.thermostat = s->thermostat;
  c.inv_tau2 = (s->thermostat && s->tau > 0 && std::isfinite(s->tau)) ? 1.0 / (s->tau * s->tau) : 0.0;
  const double hs = 0.5 * s->skin;
  c.half_skin2 = hs * hs;
  c.g = 3.0 * s->n - 3.0;
  for (int t = 0; t < kMaxTypes; ++t) {
    c.mass[t] = s->mass[t];
    c.inv_mass[t] = (float)(1.0 / s->mass[t]);
  }
  c.pt.rcc2 = s->coulomb ? (float)(s->rcc * s->rcc) : 0.0f;
  c.pt.inv_rcc2 = s->coulomb ? (float)(1.0 / (s->rcc * s->rcc)) : 0.0f;
  c.pt.two_inv_rcc = s->coulomb ? (float)(2.0 / s->rcc) : 0.0f;
  for (int a = 0; a < s->ntypes * s->ntypes; ++a) {
    // listed within the larger of the two cutoffs of the pair, plus the skin
    const double rs = (s->coulomb ? std::max(s->rc[a], s->rcc) : s->rc[a]) + s->skin;
    c.pt.qq[a] = s->coulomb ? (float)(s->charge[a / s->ntypes] * s->charge[a % s->ntypes]) : 0.0f;
    c.pt.cs2[a] = (float)(rs * rs);
    c.pt.rc2[a] = (float)(s->rc[a] * s->rc[a]);
    c.pt.sig2[a] = (float)(s->sigma[a] * s->sigma[a]);
    c.pt.eps4[a] = (float)(4.0 * s->eps[a]);
    c.pt.eps24[a] = (float)(24.0 * s->eps[a]);
    c.pt.rc[a] = (float)s->rc[a];
    c.pt.ushift[a] = s->method == SRMD_CUT_TRUNC ? 0.0f : (float)lj_u(s->rc[a], s->sigma[a], s->eps[a]);
    c.pt.fc[a] = s->method == SRMD_CUT_SF ? (float)lj_f(s->rc[a], s->sigma[a], s->eps[a]) : 0.0f;
    if (s->pot == 1) {
      const double A = s->mie_a[a], B = s->mie_b[a];
      const int m = s->mie_m[a], n = s->mie_n[a];
      c.pt.eps4[a] = (float)A;
      c.pt.eps24[a] = (float)(m * A);
      c.pt.mie_b[a] = (float)B;
      c.pt.mie_nb[a] = (float)(n * B);
      c.pt.mie_hm[a] = m / 2;
      c.pt.mie_hn[a] = n / 2;
      c.pt.ushift[a] = s->method == SRMD_CUT_TRUNC ? 0.0f : (float)mie_u(s->rc[a], A, B, m, n, s->sigma[a]);
      c.pt.fc[a] = s->method == SRMD_CUT_SF ? (float)mie_f(s->rc[a], A, B, m, n, s->sigma[a]) : 0.0f;
    }
    if (s->pot >= 2) {
      const double *q = s->gen_p[a], sg = s->sigma[a];
      double uc, fcut;
      further_uf(s->pot, q, sg, s->rc[a], &uc, &fcut);
      c.pt.eps4[a] = c.pt.eps24[a] = 0.0f;
      c.pt.ushift[a] = s->method == SRMD_CUT_TRUNC ? 0.0f : (float)uc;
      c.pt.fc[a] = s->method == SRMD_CUT_SF ? (float)fcut : 0.0f;
      float *g = c.pt.gen[a];
      if (s->pot == 2) {
        g[0] = (float)(q[0] * sg * std::exp(q[1] * sg));
        g[1] = (float)q[1];
      } else if (s->pot == 3) {
        g[0] = (float)q[0];
        g[1] = (float)(1.0 / q[1]);
        g[2] = (float)q[2];
      } else if (s->pot == 4) {
        g[0] = (float)q[0];
        g[1] = (float)(1.0 / (sg * sg));
      } else if (s->pot == 5) {
        g[0] = (float)q[0];
        g[1] = (float)(1.0 / sg);
      } else {
        g[0] = (float)q[0];
        g[1] = (float)q[1];
        g[2] = (float)(1.0 / sg);
      }
    }
  }
  return SRMD_OK;
}

// Rebuild the kernel constants, the cell grid and the list storage after any change
// of parameters or launch shape.
srmd_status prepare(srmd_system *s) {
  if (s->method < 0 || !all_pairs_given(s))
    return fail(s, SRMD_EINVAL, "pair potential not set for every type pair (srmd_set_pair_lj)");
  if (s->coulomb && (s->method != SRMD_CUT_SF || s->pot != 0))
    return fail(s, SRMD_EUNSUPPORTED, "the Coulomb term runs with shifted-force Lennard-Jones (SRMD_CUT_SF) only");
  if (!s->dirty) return SRMD_OK;
  srmd_status st0 = fill_const(s);
  if (st0 != SRMD_OK) return st0;
  SysConst &c = s->c;
  const int nmax = s->n_max;
  // storage that depends on the layout
  const long long need_nbl = (long long)nmax * c.nvp;
  if (need_nbl > s->nbl_alloc) {
    dev_free(s, s->p.nbl);
    s->p.nbl = (int *)dev_alloc(s, sizeof(int) * (size_t)need_nbl);
    if (!s->p.nbl) return fail(s, SRMD_ENOMEM, "neighbour list allocation failed");
    s->nbl_alloc = need_nbl;
  }
  if (c.ncell + 1 > s->ncell_alloc) {
    dev_free(s, s->p.cell_count);
    dev_free(s, s->p.cell_start);
    s->p.cell_count = (unsigned *)dev_alloc(s, sizeof(unsigned) * (size_t)(c.ncell + 1));
    s->p.cell_start = (unsigned *)dev_alloc(s, sizeof(unsigned) * (size_t)(c.ncell + 1));
    if (!s->p.cell_count || !s->p.cell_start) return fail(s, SRMD_ENOMEM, "cell arrays allocation failed");
    HIPCHK(s, hipMemsetAsync(s->p.cell_count, 0, sizeof(unsigned) * (size_t)(c.ncell + 1), s->stream));
    HIPCHK(s, hipMemsetAsync(s->p.cell_start, 0, sizeof(unsigned) * (size_t)(c.ncell + 1), s->stream));
    s->ncell_alloc = c.ncell + 1;
  }
  const int threads = s->tp * s->ppb;
  const int blocks = (int)(((long long)s->n * s->tp + threads - 1) / threads);
  // block partials, a second set of them and one partial per wave unit (the
  // persistent kernel alternates the two sets of block partials by step parity)
  const int nparts = 2 * blocks + blocks * (threads / 64);
  if (nparts > s->part_alloc) {
    dev_free(s, s->p.part);
    s->p.part = (BlockPartial *)dev_alloc(s, sizeof(BlockPartial) * (size_t)nparts);
    if (!s->p.part) return fail(s, SRMD_ENOMEM, "partials allocation failed");
    s->part_alloc = nparts;
  }
  resolve_persistent(s);
  drop_graphs(s);
  s->dirty = false;
  return request_rebuild(s);
}


// The step kernel ends the step itself (its last workgroup runs the reduction,
// thermostat and record, and a small system's sort) when asked to, when its
// workgroups are whole waves and when the sort's arrays fit the LDS of a launch.
// How a launch-chain step ends and builds its list: 0 the separate end-of-step
// kernel; 1 the step kernel's last workgroup ends the step; 2 as 1, and a small
// system's wave-builder or all-pairs lists are built at the start of the step
// kernel (no list kernel in the chain) when each wave has at most kBuildPerWave
// (all pairs: kBuildPerWaveAllPairs) particles to build.
int step_tail(const srmd_system *s) {
  const int threads = s->tp * s->ppb;
  if (s->tail_req == 0 || threads % 64 != 0 || tail_lds_bytes(s->c, threads, 1) > kTailLdsMax) return 0;
  // automatic: not for a small system's grid of more than 256 workgroups, which all
  // end at about the same time and queue on the arrival counters (measured slower)
  if (s->tail_req < 0 && s->c.small_sort && step_blocks(s) > kTailAutoBlocks) return 0;
  const int per_wave = s->c.list_kind == 4 ? kBuildPerWaveAllPairs : kBuildPerWave;
  if (s->tail_req != 1 && s->c.small_sort && (s->c.list_kind == 1 || s->c.list_kind == 4) &&
      s->ppb <= per_wave * (threads / 64) &&
      tail_lds_bytes(s->c, threads, 2) <= kTailLdsMax)
    return 2;
  return 1;
}

// Enqueue one launch-chain step on position buffer cb.
hipError_t enqueue_step(srmd_system *s, int cb) {
  const int tail = step_tail(s);
  hipError_t e = tail == 2 ? hipSuccess : launch_rebuild(s->stream, s->c, s->p, cb);
  if (e == hipSuccess)
    e = launch_step(s->tp, kmethod(s), (int)s->prec, step_blocks(s), s->tp * s->ppb, s->stream, s->c, s->p, cb,
                    tail, tail ? tail_lds_bytes(s->c, s->tp * s->ppb, tail) : 0);
  if (e == hipSuccess && !tail) e = launch_finish(0, step_blocks(s), cb ^ 1, s->stream, s->c, s->p);
  return e;
}

srmd_status enqueue_steps(srmd_system *s, int count, int cur) {
  for (int k = 0; k < count; ++k) HIPCHK(s, enqueue_step(s, (cur + k) & 1));
  return SRMD_OK;
}

srmd_status get_graph(srmd_system *s, int count, int cur, hipGraphExec_t *out) {
  auto key = std::make_pair(count, cur);
  auto it = s->graphs.find(key);
  if (it != s->graphs.end()) {
    *out = it->second;
    return SRMD_OK;
  }
  hipGraph_t g;
  HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  srmd_status st = enqueue_steps(s, count, cur);
  hipGraph_t g2 = nullptr;
  hipError_t e = hipStreamEndCapture(s->stream, &g2);
  if (st != SRMD_OK) {
    if (g2) (void)hipGraphDestroy(g2);
    return st;
  }
  if (e != hipSuccess) return fail(s, SRMD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  g = g2;
  hipGraphExec_t ge;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(s, SRMD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  s->graphs[key] = ge;
  *out = ge;
  return SRMD_OK;
}

srmd_status alloc_snapshot(srmd_system *s) {
  if (s->snap.pos) return SRMD_OK;
  const size_t n = (size_t)s->n;
  Snapshot &q = s->snap;
  q.pos = (float4 *)dev_alloc(s, sizeof(float4) * n);
  q.vel = (float4 *)dev_alloc(s, sizeof(float4) * n);
  q.last = (float4 *)dev_alloc(s, sizeof(float4) * n);
  q.img = (int4 *)dev_alloc(s, sizeof(int4) * n);
  q.ctl = (Control *)dev_alloc(s, sizeof(Control));
  if (s->prec == SRMD_PREC_F64POS) q.pos64 = (double *)dev_alloc(s, sizeof(double) * 3 * n);
  if (s->prec == SRMD_PREC_F32_KAHAN) q.kahan = (float4 *)dev_alloc(s, sizeof(float4) * n);
  if (!q.pos || !q.vel || !q.last || !q.img || !q.ctl || (s->p.pos64 && !q.pos64) || (s->p.kahan && !q.kahan)) {
    for (void *b : {(void *)q.pos, (void *)q.vel, (void *)q.last, (void *)q.img, (void *)q.ctl, (void *)q.pos64,
                    (void *)q.kahan})
      dev_free(s, b);
    q = Snapshot{};
    return fail(s, SRMD_ENOMEM, "snapshot allocation failed");
  }
  return SRMD_OK;
}

// Put the call-start snapshot back (after a list overflow).
srmd_status restore_snapshot(srmd_system *s) {
  const size_t n = (size_t)s->n;
  const Snapshot &q = s->snap;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->stream);
  };
  HIPCHK(s, cp(s->p.pos[s->cur], q.pos, sizeof(float4) * n));
  HIPCHK(s, cp(s->p.vel, q.vel, sizeof(float4) * n));
  HIPCHK(s, cp(s->p.last, q.last, sizeof(float4) * n));
  HIPCHK(s, cp(s->p.img, q.img, sizeof(int4) * n));
  HIPCHK(s, cp(s->p.ctl, q.ctl, sizeof(Control)));
  if (s->p.pos64) HIPCHK(s, cp(s->p.pos64, q.pos64, sizeof(double) * 3 * n));
  if (s->p.kahan) HIPCHK(s, cp(s->p.kahan, q.kahan, sizeof(float4) * n));
  return SRMD_OK;
}

srmd_status read_ctl(srmd_system *s, Control *h) {
  HIPCHK(s, hipMemcpyAsync(h, s->p.ctl, sizeof(Control), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

// Double the list capacity after an overflow (paper section 4: re-allocation with
// doubled capacity) and mark the layout for rebuild.
srmd_status regrow(srmd_system *s) {
  s->n_max = std::min(2 * s->n_max, (s->n + 63) / 64 * 64);
  s->dirty = true;
  return prepare(s);
}

// After a persistent launch: report a grid barrier that timed out (error bit 2) and
// clear the bit (the arrival words are cleared before every launch).
srmd_status check_barrier(srmd_system *s, Control *h) {
  if (!(h->error & 4)) return SRMD_OK;
  h->error &= ~4;
  srmd_status st = h2d_sync(s, s->p.ctl, h, sizeof(Control));
  if (st != SRMD_OK) return st;
  return fail(s, SRMD_EHIP, "persistent kernel: a device-wide barrier timed out");
}

// The descriptor of this system for a persistent launch.
ReplicaDesc make_desc(const srmd_system *s) {
  ReplicaDesc d;
  std::memset(&d, 0, sizeof(d));
  d.c = s->c;
  d.p = s->p;
  d.cur = s->cur;
  d.G = step_blocks(s);
  d.vb = s->tp * s->ppb;
  return d;
}

// One launch of the persistent kernel over cnt steps: the system split over
// persist_groups workgroups (job w of g on workgroup w).
srmd_status launch_persistent(srmd_system *s, int cnt) {
  const int g = s->persist_groups;
  if (g > s->jobs_cap) {
    dev_free(s, s->d_jobs);
    dev_free(s, s->d_job_off);
    s->d_jobs = (CoopJob *)dev_alloc(s, sizeof(CoopJob) * (size_t)g);
    s->d_job_off = (int *)dev_alloc(s, sizeof(int) * (size_t)(g + 1));
    if (!s->d_jobs || !s->d_job_off) return fail(s, SRMD_ENOMEM, "persistent job table allocation failed");
    s->jobs_cap = g;
    s->jobs_g = 0;
  }
  if (g != s->jobs_g) {
    std::vector<CoopJob> hj((size_t)g);
    std::vector<int> ho((size_t)g + 1);
    for (int w = 0; w < g; ++w) hj[(size_t)w] = CoopJob{0, w, g, 0};
    for (int w = 0; w <= g; ++w) ho[(size_t)w] = w;
    HIPCHK(s, hipMemcpyAsync(s->d_jobs, hj.data(), sizeof(CoopJob) * hj.size(), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->d_job_off, ho.data(), sizeof(int) * ho.size(), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->jobs_g = g;
  }
  if (!s->d_desc) {
    s->d_desc = (ReplicaDesc *)dev_alloc(s, sizeof(ReplicaDesc));
    if (!s->d_desc) return fail(s, SRMD_ENOMEM, "persistent descriptor allocation failed");
    s->desc_valid = false;
  }
  const ReplicaDesc d = make_desc(s);
  if (!s->desc_valid || std::memcmp(&d, &s->host_desc, sizeof(d)) != 0) {
    s->host_desc = d;
    HIPCHK(s, hipMemcpyAsync(s->d_desc, &s->host_desc, sizeof(ReplicaDesc), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->desc_valid = true;
  }
  if (g > 1) HIPCHK(s, hipMemsetAsync(s->p.bar_flags, 0, sizeof(unsigned) * 2 * 256, s->stream));
  HIPCHK(s, launch_multi(s->tp, kmethod(s), !s->c.small_sort, g, persist_lds(s), s->stream, s->d_desc, s->d_jobs, s->d_job_off,
                         cnt, g > 1));
  s->cur ^= (cnt & 1);
  return SRMD_OK;
}

// Persistent mode runs kPersistChunk steps per launch: launches stay short, and the
// per-launch cost (a few microseconds) is spread over hundreds of steps.
srmd_status run_persistent(srmd_system *s, long long nsteps) {
  long long left = nsteps;
  while (left > 0) {
    const int cnt = (int)std::min<long long>(left, kPersistChunk);
    srmd_status st = launch_persistent(s, cnt);
    if (st != SRMD_OK) return st;
    left -= cnt;
  }
  return SRMD_OK;
}

srmd_status run_steps(srmd_system *s, long long nsteps) {
  srmd_status st0 = flush_host_sort(s);
  if (st0 != SRMD_OK) return st0;
  if (!s->persist_err.empty()) return fail(s, SRMD_EUNSUPPORTED, s->persist_err);
  if (s->persist_groups > 0) return run_persistent(s, nsteps);
  long long left = nsteps;
  while (left > 0) {
    const int cnt = (int)std::min<long long>(left, kChunk);
    hipGraphExec_t ge;
    srmd_status st = get_graph(s, cnt, s->cur, &ge);
    if (st != SRMD_OK) return st;
    HIPCHK(s, hipGraphLaunch(ge, s->stream));
    s->cur ^= (cnt & 1);
    left -= cnt;
  }
  return SRMD_OK;
}

void to_public(const Thermo &t, srmd_thermo *o) {
  o->pe = t.pe;
  o->ke = t.ke;
  o->virial = t.virial;
  o->temperature = t.temperature;
  o->pressure = t.pressure;
  o->xi = t.xi;
  o->xi_integral = t.xi_integral;
  o->h_conserved = t.h_conserved;
  o->ke_half = t.ke_half;
  o->step = t.step;
  o->n_rebuilds = t.n_rebuilds;
  o->max_nbrs = t.max_nbrs;
  o->reserved = 0;
}

float wrap_f32(double x, double L) {
  double y = x - L * std::floor(x / L + 0.5);
  float f = (float)y;
  const float h = 0.5f * (float)L;
  if (f >= h) f -= (float)L;
  if (f < -h) f += (float)L;
  return f;
}

// Upload positions / velocities given in original order; ids become the identity.
srmd_status upload_state(srmd_system *s, const float *pos, const float *vel, const int32_t *type) {
  const int n = s->n;
  std::vector<float4> hp((size_t)n), hv((size_t)n);
  std::vector<int4> hi((size_t)n);
  std::vector<double> h64;
  if (s->prec == SRMD_PREC_F64POS) h64.resize(3 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    float x[3];
    for (int k = 0; k < 3; ++k) x[k] = wrap_f32((double)pos[3 * i + k], (double)s->Lf[k]);
    int ty = type[i];
    float w;
    std::memcpy(&w, &ty, 4);
    hp[(size_t)i] = make_float4(x[0], x[1], x[2], w);
    hv[(size_t)i] = vel ? make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    hi[(size_t)i] = make_int4(0, 0, 0, i);
    if (!h64.empty())
      for (int k = 0; k < 3; ++k) h64[3 * (size_t)i + k] = (double)x[k];
  }
  HIPCHK(s, hipMemcpyAsync(s->p.pos[s->cur], hp.data(), sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.last, hp.data(), sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.vel, hv.data(), sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.img, hi.data(), sizeof(int4) * (size_t)n, hipMemcpyHostToDevice, s->stream));
  if (s->p.pos64)
    HIPCHK(s, hipMemcpyAsync(s->p.pos64, h64.data(), sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, s->stream));
  if (s->p.kahan) HIPCHK(s, hipMemsetAsync(s->p.kahan, 0, sizeof(float4) * (size_t)n, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

// A copy of the dynamic state in host memory (the autotuner's stored configuration).
struct HostState {
  int cur = 0;
  std::vector<float4> pos, vel, last, kahan;
  std::vector<int4> img;
  std::vector<double> pos64;
  Control ctl;
  Thermo thermo;
};

srmd_status save_host_state(srmd_system *s, HostState *h) {
  const size_t n = (size_t)s->n;
  h->cur = s->cur;
  h->pos.resize(n);
  h->vel.resize(n);
  h->last.resize(n);
  h->img.resize(n);
  HIPCHK(s, hipMemcpyAsync(h->pos.data(), s->p.pos[s->cur], sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(h->vel.data(), s->p.vel, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(h->last.data(), s->p.last, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(h->img.data(), s->p.img, sizeof(int4) * n, hipMemcpyDeviceToHost, s->stream));
  if (s->p.pos64) {
    h->pos64.resize(3 * n);
    HIPCHK(s, hipMemcpyAsync(h->pos64.data(), s->p.pos64, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s->stream));
  }
  if (s->p.kahan) {
    h->kahan.resize(n);
    HIPCHK(s, hipMemcpyAsync(h->kahan.data(), s->p.kahan, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHK(s, hipMemcpyAsync(&h->ctl, s->p.ctl, sizeof(Control), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(&h->thermo, s->p.thermo, sizeof(Thermo), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

// Put a stored state back; the list is rebuilt before the next force evaluation.
srmd_status restore_host_state(srmd_system *s, const HostState &h) {
  const size_t n = (size_t)s->n;
  s->cur = h.cur;
  HIPCHK(s, hipMemcpyAsync(s->p.pos[s->cur], h.pos.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.vel, h.vel.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.last, h.last.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.img, h.img.data(), sizeof(int4) * n, hipMemcpyHostToDevice, s->stream));
  if (s->p.pos64 && !h.pos64.empty())
    HIPCHK(s, hipMemcpyAsync(s->p.pos64, h.pos64.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, s->stream));
  if (s->p.kahan && !h.kahan.empty())
    HIPCHK(s, hipMemcpyAsync(s->p.kahan, h.kahan.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
  Control c = h.ctl;
  c.rebuild = 1;
  HIPCHK(s, hipMemcpyAsync(s->p.ctl, &c, sizeof(Control), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.thermo, &h.thermo, sizeof(Thermo), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->sort_pending = true;
  return SRMD_OK;
}

srmd_status ensure_trace(srmd_system *s, long long cap) {
  if (cap <= s->trace_alloc) return SRMD_OK;
  dev_free(s, s->p.trace);
  s->p.trace = (Thermo *)dev_alloc(s, sizeof(Thermo) * (size_t)cap);
  if (!s->p.trace) return fail(s, SRMD_ENOMEM, "trace allocation failed");
  s->trace_alloc = cap;
  // the pointer is baked into the captured graphs (the persistent and batch
  // descriptors are compared with the system before every launch); the list and
  // the trajectory do not depend on the trace, so no rebuild is requested
  drop_graphs(s);
  return SRMD_OK;
}

}  // namespace

struct srmd_batch {
  std::vector<srmd_system *> sys;
  std::vector<ReplicaDesc> host_desc;
  ReplicaDesc *d_desc = nullptr;
  DevBuf desc_buf, jobs_buf, joboff_buf;  // device tables, from the allocator hook
  std::vector<CoopJob> jobs;     // per workgroup, in replica order
  std::vector<int> job_off;      // workgroup b runs jobs[job_off[b] .. job_off[b + 1])
  std::vector<int> pieces;       // workgroups of each replica
  CoopJob *d_jobs = nullptr;
  int *d_job_off = nullptr;
  int nwg = 0;
  bool cooperative = false;      // some replica is split over several workgroups
  hipStream_t stream = nullptr;
  int tp = 0, method = 0;
  size_t lds = 0;
  int max_wg = 0;                // the caller's workgroup limit (0: none)
  std::string err;
};

namespace {

srmd_status bfail(srmd_batch *b, srmd_status st, const std::string &msg) {
  if (b) b->err = msg;
  g_thread_error = msg;
  return st;
}

// Refresh the replica descriptors from the systems (constants, pointers, buffers).
srmd_status batch_sync_desc(srmd_batch *b) {
  bool changed = false;
  for (size_t r = 0; r < b->sys.size(); ++r) {
    srmd_system *s = b->sys[r];
    srmd_status st = prepare(s);
    if (st != SRMD_OK) return bfail(b, st, std::string("replica ") + std::to_string(r) + ": " + s->err);
    if (s->tp != b->tp || kmethod(s) != b->method)
      return bfail(b, SRMD_EINVAL, "replicas must share the cutoff method and the threads per particle");
    const ReplicaDesc d = make_desc(s);
    if (std::memcmp(&d, &b->host_desc[r], sizeof(d)) != 0) {
      b->host_desc[r] = d;
      changed = true;
    }
  }
  if (changed) {
    hipError_t e = hipMemcpyAsync(b->d_desc, b->host_desc.data(), sizeof(ReplicaDesc) * b->host_desc.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, SRMD_EHIP, std::string("descriptor upload: ") + hipGetErrorString(e));
  }
  return SRMD_OK;
}

// Longest-processing-time packing of items (loads) into nb bins: largest first, each
// on the least-loaded bin that still takes a job.  Returns the largest bin load, or
// a negative value if some item found no bin.
double lpt_pack(const std::vector<std::pair<double, int>> &items, int nb, int max_jobs,
                std::vector<std::vector<int>> *bins) {
  std::vector<double> load((size_t)nb, 0.0);
  if (bins) bins->assign((size_t)nb, {});
  std::vector<int> count((size_t)nb, 0);
  for (const auto &it : items) {
    int best = -1;
    for (int q = 0; q < nb; ++q)
      if (count[(size_t)q] < max_jobs && (best < 0 || load[(size_t)q] < load[(size_t)best])) best = q;
    if (best < 0) return -1.0;
    load[(size_t)best] += it.first;
    count[(size_t)best] += 1;
    if (bins) (*bins)[(size_t)best].push_back(it.second);
  }
  double m = 0.0;
  for (double l : load) m = std::max(m, l);
  return m;
}

// Distribute the replicas over at most W workgroups.  The work of a piece is taken as
// its particle count plus a fixed cost per step (kJobCost for a whole replica,
// kPieceCost for a piece of a split one: its grid barrier and its full position
// load), in particle equivalents.  A replica is either whole, sharing a workgroup
// with other whole replicas (run one after the other), or split into g_r > 1
// pieces, each alone on its workgroup (its grid barriers then never wait behind
// other work).  Starting from all replicas whole, the replica with the largest piece
// is split one piece further while workgroups remain; the whole replicas go to the
// remaining workgroups by longest-processing-time packing; the configuration with
// the smallest largest load is kept.
constexpr double kJobCost = 50.0, kPieceCost = 150.0;

srmd_status batch_plan(srmd_batch *b, int W) {
  const int R = (int)b->sys.size();
  std::vector<int> g((size_t)R, 1), best_g;
  double best = -1.0;
  std::vector<int> order((size_t)R);
  for (int r = 0; r < R; ++r) order[(size_t)r] = r;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->sys[(size_t)a]->n > b->sys[(size_t)c]->n; });
  for (int it = 0; it <= 2 * W; ++it) {
    int used = 0;
    double split_max = 0.0;
    std::vector<std::pair<double, int>> whole;
    for (int r : order) {
      const double n = b->sys[(size_t)r]->n;
      if (g[(size_t)r] > 1) {
        used += g[(size_t)r];
        split_max = std::max(split_max, n / g[(size_t)r] + kPieceCost);
      } else {
        whole.push_back({n + kJobCost, r});
      }
    }
    const int free_wg = W - used;
    if (free_wg < 0 || (free_wg < 1 && !whole.empty())) break;
    const double packed = whole.empty() ? 0.0 : lpt_pack(whole, free_wg, multi_max_jobs(), nullptr);
    if (packed >= 0.0) {
      const double mk = std::max(split_max, packed);
      if (best < 0.0 || mk < best) {
        best = mk;
        best_g = g;
      }
    }
    // split the replica with the largest piece one piece further
    int rmax = -1;
    double pmax = 0.0;
    for (int r = 0; r < R; ++r) {
      const srmd_system *s = b->sys[(size_t)r];
      if (g[(size_t)r] >= std::min({step_blocks(s), 256, W})) continue;
      const double piece = (double)s->n / g[(size_t)r];
      if (piece > pmax) {
        pmax = piece;
        rmax = r;
      }
    }
    if (rmax < 0) break;
    g[(size_t)rmax] += 1;
  }
  if (best < 0.0) return bfail(b, SRMD_EUNSUPPORTED, "too many replicas for the workgroups of one launch");
  b->pieces = best_g;
  std::vector<std::vector<CoopJob>> per;
  std::vector<std::pair<double, int>> whole;
  for (int r : order) {
    if (best_g[(size_t)r] > 1)
      for (int w = 0; w < best_g[(size_t)r]; ++w) per.push_back({CoopJob{r, w, best_g[(size_t)r], 0}});
    else
      whole.push_back({(double)b->sys[(size_t)r]->n + kJobCost, r});
  }
  if (!whole.empty()) {
    std::vector<std::vector<int>> bins;
    const int free_wg = W - (int)per.size();
    lpt_pack(whole, std::min(free_wg, (int)whole.size()), multi_max_jobs(), &bins);
    for (auto &bin : bins) {
      std::vector<CoopJob> v;
      for (int r : bin) v.push_back(CoopJob{r, 0, 1, 0});
      std::sort(v.begin(), v.end(), [](const CoopJob &a, const CoopJob &c) { return a.rep < c.rep; });
      if (!v.empty()) per.push_back(v);
    }
  }
  b->jobs.clear();
  b->job_off.assign(1, 0);
  b->cooperative = false;
  for (auto &v : per) {
    for (const CoopJob &j : v) {
      b->jobs.push_back(j);
      b->cooperative = b->cooperative || j.g > 1;
    }
    b->job_off.push_back((int)b->jobs.size());
  }
  b->nwg = (int)per.size();
  // the tables of an earlier plan are released once no launch can still read them
  if (b->jobs_buf.ptr || b->joboff_buf.ptr) {
    (void)hipStreamSynchronize(b->stream);
    raw_free(b->jobs_buf);
    raw_free(b->joboff_buf);
  }
  b->jobs_buf = raw_alloc(sizeof(CoopJob) * b->jobs.size());
  b->joboff_buf = raw_alloc(sizeof(int) * b->job_off.size());
  b->d_jobs = (CoopJob *)b->jobs_buf.ptr;
  b->d_job_off = (int *)b->joboff_buf.ptr;
  if (!b->d_jobs || !b->d_job_off) return bfail(b, SRMD_ENOMEM, "batch job tables: allocation failed");
  hipError_t e = hipMemcpyAsync(b->d_jobs, b->jobs.data(), sizeof(CoopJob) * b->jobs.size(), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_job_off, b->job_off.data(), sizeof(int) * b->job_off.size(), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, SRMD_EHIP, std::string("batch job tables: ") + hipGetErrorString(e));
  return SRMD_OK;
}

// Descriptors and workgroup plan of the batch for the systems' current launch shapes
// (all replicas share b->tp).
srmd_status batch_replan(srmd_batch *b) {
  srmd_status st = batch_sync_desc(b);
  if (st != SRMD_OK) return st;
  int W = multi_max_groups(b->tp, b->method, false, b->lds);
  if (b->max_wg > 0) W = std::min(W, b->max_wg);
  if (W < 1) return bfail(b, SRMD_EUNSUPPORTED, "the persistent kernel does not fit on the device");
  return batch_plan(b, W);
}

// Put the call-start snapshot back after a list overflow (cur0: the position
// buffer in use at the call start), clear the overflow bit and double the list
// capacity (paper section 4); the next run rebuilds the list.
srmd_status restore_and_regrow(srmd_system *s, int cur0) {
  s->cur = cur0;
  srmd_status st = restore_snapshot(s);
  if (st != SRMD_OK) return st;
  Control r;
  st = read_ctl(s, &r);
  if (st != SRMD_OK) return st;
  r.error &= ~2;
  st = h2d_sync(s, s->p.ctl, &r, sizeof(Control));
  if (st != SRMD_OK) return st;
  return regrow(s);
}

// nsteps steps of one system with list-overflow recovery: the call-start state is
// kept in a device snapshot; a run whose list overflowed is restored, its capacity
// doubled, and replayed, so the trajectory is that of a list that never overflowed.
// Trace settings live in the control block so the captured graphs stay valid.
srmd_status run_with_replay(srmd_system *s, long long nsteps, int32_t thermo_every, long long cap) {
  for (int attempt = 0; attempt < 8; ++attempt) {
    const int cur0 = s->cur;
    HIPCHK(s, launch_call_begin(s->stream, s->c, s->p, s->snap, s->cur, thermo_every, cap));
    srmd_status st = run_steps(s, nsteps);
    if (st != SRMD_OK) return st;
    // the one host round trip of the call: the control block's sticky error word
    HIPCHK(s, hipMemcpyAsync(s->h_ctl, s->p.ctl, sizeof(Control), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    Control h = *s->h_ctl;
    st = check_barrier(s, &h);
    if (st != SRMD_OK) return st;
    if (h.error & 2) {
      st = restore_and_regrow(s, cur0);
      if (st != SRMD_OK) return st;
      continue;
    }
    if (h.error & 1) return fail(s, SRMD_ESTATE, "non-finite force or position during the run");
    return SRMD_OK;
  }
  return fail(s, SRMD_ENOMEM, "neighbour list kept overflowing");
}

// Copy the records of the last run's device trace into trace (cap entries at most).
srmd_status download_trace(srmd_system *s, long long cap, srmd_thermo *trace) {
  if (cap <= 0) return SRMD_OK;
  const long long nrec = s->h_ctl->n_records;  // read back at the end of the run
  if (nrec <= 0) return SRMD_OK;
  std::vector<Thermo> tmp((size_t)std::min<long long>(nrec, cap));
  HIPCHK(s, hipMemcpyAsync(tmp.data(), s->p.trace, sizeof(Thermo) * tmp.size(), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (size_t k = 0; k < tmp.size(); ++k) to_public(tmp[k], &trace[k]);
  return SRMD_OK;
}

}  // namespace

// ====================================================================== C-ABI

extern "C" {

const char *srmd_last_error(const srmd_system *s) { return s ? s->err.c_str() : g_thread_error.c_str(); }

srmd_status srmd_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
  if (alloc && !free_fn) return fail(nullptr, SRMD_EINVAL, "allocator hook needs both alloc and free");
  g_alloc.alloc = alloc;
  g_alloc.free_fn = alloc ? free_fn : nullptr;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return SRMD_OK;
}

srmd_status srmd_create(srmd_system **out, int32_t n, int32_t ntypes, const double box[3], const float *pos,
                        const int32_t *type, const float *vel, const double *mass, srmd_precision prec,
                        void *hip_stream) {
  if (!out) return fail(nullptr, SRMD_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 2) return fail(nullptr, SRMD_EINVAL, "need at least 2 particles");
  if (ntypes < 1 || ntypes > kMaxTypes) return fail(nullptr, SRMD_EINVAL, "ntypes must be in 1..4");
  if (!box || !pos || !type) return fail(nullptr, SRMD_EINVAL, "box, pos and type are required");
  if (prec != SRMD_PREC_F32 && prec != SRMD_PREC_F32_KAHAN && prec != SRMD_PREC_F64POS)
    return fail(nullptr, SRMD_EINVAL, "unknown precision");
  for (int k = 0; k < 3; ++k)
    if (!(box[k] > 0) || !std::isfinite(box[k]) || !std::isfinite((float)box[k]))
      return fail(nullptr, SRMD_EINVAL, "box sides must be positive and finite");
  for (long long i = 0; i < 3LL * n; ++i) {
    if (!std::isfinite(pos[i])) return fail(nullptr, SRMD_EINVAL, "non-finite position");
    if (vel && !std::isfinite(vel[i])) return fail(nullptr, SRMD_EINVAL, "non-finite velocity");
  }
  for (int i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= ntypes) return fail(nullptr, SRMD_EINVAL, "particle type out of range");
  if (mass)
    for (int t = 0; t < ntypes; ++t)
      if (!(mass[t] > 0) || !std::isfinite(mass[t])) return fail(nullptr, SRMD_EINVAL, "masses must be positive");
  srmd_system *s = new (std::nothrow) srmd_system();
  if (!s) return fail(nullptr, SRMD_ENOMEM, "host allocation failed");
  s->n = n;
  s->ntypes = ntypes;
  s->prec = prec;
  for (int k = 0; k < 3; ++k) s->Lf[k] = (float)box[k];
  if (mass)
    for (int t = 0; t < ntypes; ++t) s->mass[t] = mass[t];
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return fail(nullptr, SRMD_EHIP, "hipStreamCreate failed");
    }
    s->own_stream = true;
  }
  if (hipHostMalloc((void **)&s->h_ctl, sizeof(Control), hipHostMallocDefault) != hipSuccess) {
    s->h_ctl = nullptr;
    srmd_destroy(s);
    return fail(nullptr, SRMD_ENOMEM, "pinned host allocation failed");
  }
  const size_t N = (size_t)n;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void *q = dev_alloc(s, bytes);
    ok = ok && q;
    return q;
  };
  s->p.pos[0] = (float4 *)A(sizeof(float4) * N);
  s->p.pos[1] = (float4 *)A(sizeof(float4) * N);
  s->p.vel = (float4 *)A(sizeof(float4) * N);
  s->p.img = (int4 *)A(sizeof(int4) * N);
  s->p.force = (float4 *)A(sizeof(float4) * N);
  s->p.wpart = (float *)A(sizeof(float) * N);
  s->p.last = (float4 *)A(sizeof(float4) * N);
  s->p.nnb = (int *)A(sizeof(int) * N);
  s->p.cell_of = (unsigned *)A(sizeof(unsigned) * N);
  s->p.slot_in_cell = (unsigned *)A(sizeof(unsigned) * N);
  s->p.perm_tmp = (unsigned *)A(sizeof(unsigned) * N);
  s->p.t_pos = (float4 *)A(sizeof(float4) * N);
  s->p.t_vel = (float4 *)A(sizeof(float4) * N);
  s->p.t_img = (int4 *)A(sizeof(int4) * N);
  s->p.ctl = (Control *)A(sizeof(Control));
  s->p.thermo = (Thermo *)A(sizeof(Thermo));
  s->p.bar_flags = (unsigned *)A(sizeof(unsigned) * 2 * 256);
  s->p.arrive = (unsigned *)A(arrive_bytes());
  s->p.tile_count = (unsigned *)A(sizeof(unsigned) * kScanMaxTiles);
  if (prec == SRMD_PREC_F64POS) {
    s->p.pos64 = (double *)A(sizeof(double) * 3 * N);
    s->p.t_pos64 = (double *)A(sizeof(double) * 3 * N);
  }
  if (prec == SRMD_PREC_F32_KAHAN) {
    s->p.kahan = (float4 *)A(sizeof(float4) * N);
    s->p.t_kahan = (float4 *)A(sizeof(float4) * N);
  }
  if (!ok) {
    srmd_destroy(s);
    return fail(nullptr, SRMD_ENOMEM, "device allocation failed");
  }
  Control hc;
  std::memset(&hc, 0, sizeof(hc));
  hc.rebuild = 1;
  Thermo ht;
  std::memset(&ht, 0, sizeof(ht));
  if (hipMemcpyAsync(s->p.ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipMemcpyAsync(s->p.thermo, &ht, sizeof(ht), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.force, 0, sizeof(float4) * N, s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.wpart, 0, sizeof(float) * N, s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.nnb, 0, sizeof(int) * N, s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.tile_count, 0, sizeof(unsigned) * kScanMaxTiles, s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.arrive, 0, arrive_bytes(), s->stream) != hipSuccess ||
      hipMemsetAsync(s->p.t_pos, 0, sizeof(float4) * N, s->stream) != hipSuccess) {
    srmd_destroy(s);
    return fail(nullptr, SRMD_EHIP, "initial upload failed");
  }
  srmd_status st = upload_state(s, pos, vel, type);
  if (st != SRMD_OK) {
    std::string m = s->err;
    srmd_destroy(s);
    return fail(nullptr, st, m);
  }
  *out = s;
  return SRMD_OK;
}

srmd_status srmd_destroy(srmd_system *s) {
  if (!s) return SRMD_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);
  while (!s->bufs.empty()) dev_free(s, s->bufs.back().ptr);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  if (s->h_ctl) (void)hipHostFree(s->h_ctl);
  delete s;
  return SRMD_OK;
}

srmd_status srmd_set_pair_lj(srmd_system *s, int32_t ti, int32_t tj, double sigma, double epsilon, double rcut,
                             srmd_cutoff method) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (ti < 0 || tj < 0 || ti >= s->ntypes || tj >= s->ntypes) return fail(s, SRMD_EINVAL, "type index out of range");
  if (!(sigma > 0) || !(epsilon >= 0) || !(rcut > 0) || !std::isfinite(sigma) || !std::isfinite(epsilon) ||
      !std::isfinite(rcut))
    return fail(s, SRMD_EINVAL, "sigma, rcut must be positive and epsilon non-negative");
  if (method != SRMD_CUT_TRUNC && method != SRMD_CUT_SP && method != SRMD_CUT_SF)
    return fail(s, SRMD_EINVAL, "unknown cutoff method");
  if (s->method >= 0 && s->method != (int)method)
    return fail(s, SRMD_EINVAL, "all type pairs must use the same cutoff method");
  if (s->pot >= 1) return fail(s, SRMD_EINVAL, "all type pairs must use the same potential (another one set before)");
  for (int k = 0; k < 3; ++k)
    if (!(rcut + s->skin < 0.5 * (double)s->Lf[k]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
  s->method = (int)method;
  s->pot = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int a = pass ? pair_index(s, tj, ti) : pair_index(s, ti, tj);
    s->sigma[a] = sigma;
    s->eps[a] = epsilon;
    s->rc[a] = rcut;
    s->pair_given[a] = true;
  }
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_pair_mie(srmd_system *s, int32_t ti, int32_t tj, double A, double B, int32_t m, int32_t n,
                              double sigma, double rcut, srmd_cutoff method) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (ti < 0 || tj < 0 || ti >= s->ntypes || tj >= s->ntypes) return fail(s, SRMD_EINVAL, "type index out of range");
  if (!(A >= 0) || !(B >= 0) || !std::isfinite(A) || !std::isfinite(B) || !(sigma > 0) || !std::isfinite(sigma) ||
      !(rcut > 0) || !std::isfinite(rcut))
    return fail(s, SRMD_EINVAL, "A, B must be non-negative and sigma, rcut positive");
  if (m % 2 || n % 2 || n < 2 || m <= n || m > 48)
    return fail(s, SRMD_EINVAL, "exponents must be even with 2 <= n < m <= 48");
  if (method != SRMD_CUT_TRUNC && method != SRMD_CUT_SP && method != SRMD_CUT_SF)
    return fail(s, SRMD_EINVAL, "unknown cutoff method");
  if (s->method >= 0 && s->method != (int)method)
    return fail(s, SRMD_EINVAL, "all type pairs must use the same cutoff method");
  if (s->pot == 0 || s->pot >= 2) return fail(s, SRMD_EINVAL, "all type pairs must use the same potential (another one set before)");
  for (int k = 0; k < 3; ++k)
    if (!(rcut + s->skin < 0.5 * (double)s->Lf[k]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
  s->method = (int)method;
  s->pot = 1;
  for (int pass = 0; pass < 2; ++pass) {
    const int a = pass ? pair_index(s, tj, ti) : pair_index(s, ti, tj);
    s->sigma[a] = sigma;
    s->eps[a] = 0.0;
    s->rc[a] = rcut;
    s->mie_a[a] = A;
    s->mie_b[a] = B;
    s->mie_m[a] = m;
    s->mie_n[a] = n;
    s->pair_given[a] = true;
  }
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_pair_potential(srmd_system *s, int32_t ti, int32_t tj, srmd_potential kind,
                                    const double *params, double sigma, double rcut, srmd_cutoff method) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (ti < 0 || tj < 0 || ti >= s->ntypes || tj >= s->ntypes) return fail(s, SRMD_EINVAL, "type index out of range");
  const int k = (int)kind;
  if (k < SRMD_POT_YUKAWA || k > SRMD_POT_GIRIFALCO) return fail(s, SRMD_EINVAL, "unknown potential kind");
  if (!params) return fail(s, SRMD_EINVAL, "params is NULL");
  if (!(sigma > 0) || !std::isfinite(sigma) || !(rcut > 0) || !std::isfinite(rcut))
    return fail(s, SRMD_EINVAL, "sigma and rcut must be positive");
  double p[4] = {params[0], params[1], params[2], params[3]};
  for (double v : p)
    if (!std::isfinite(v)) return fail(s, SRMD_EINVAL, "parameters must be finite");
  if (k == SRMD_POT_YUKAWA && !(p[1] >= 0 && p[1] * sigma <= 60.0))
    return fail(s, SRMD_EINVAL, "Yukawa: kappa >= 0 and kappa sigma <= 60");
  if (k == SRMD_POT_BUCKINGHAM && !(p[0] >= 0 && p[1] > 0 && p[2] >= 0))
    return fail(s, SRMD_EINVAL, "Buckingham: A >= 0, rho > 0, C >= 0");
  if (k == SRMD_POT_GIRIFALCO && !(rcut > sigma))
    return fail(s, SRMD_EINVAL, "Girifalco: rcut must exceed the diameter sigma");
  if (method != SRMD_CUT_TRUNC && method != SRMD_CUT_SP && method != SRMD_CUT_SF)
    return fail(s, SRMD_EINVAL, "unknown cutoff method");
  if (s->method >= 0 && s->method != (int)method)
    return fail(s, SRMD_EINVAL, "all type pairs must use the same cutoff method");
  if (s->pot >= 0 && s->pot != k) return fail(s, SRMD_EINVAL, "all type pairs must use the same potential");
  for (int q = 0; q < 3; ++q)
    if (!(rcut + s->skin < 0.5 * (double)s->Lf[q]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
  s->method = (int)method;
  s->pot = k;
  for (int pass = 0; pass < 2; ++pass) {
    const int a = pass ? pair_index(s, tj, ti) : pair_index(s, ti, tj);
    s->sigma[a] = sigma;
    s->eps[a] = 0.0;
    s->rc[a] = rcut;
    for (int q = 0; q < 4; ++q) s->gen_p[a][q] = p[q];
    s->pair_given[a] = true;
  }
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_coulomb_sf(srmd_system *s, const double *charge, double rcut) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!charge) {
    s->coulomb = false;
    s->dirty = true;
    return SRMD_OK;
  }
  if (!(rcut > 0) || !std::isfinite(rcut)) return fail(s, SRMD_EINVAL, "the Coulomb cutoff must be positive");
  for (int t = 0; t < s->ntypes; ++t)
    if (!std::isfinite(charge[t])) return fail(s, SRMD_EINVAL, "non-finite charge");
  for (int k = 0; k < 3; ++k)
    if (!(rcut + s->skin < 0.5 * (double)s->Lf[k]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
  for (int t = 0; t < kMaxTypes; ++t) s->charge[t] = t < s->ntypes ? charge[t] : 0.0;
  s->rcc = rcut;
  s->coulomb = true;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_skin(srmd_system *s, double skin) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!(skin >= 0) || !std::isfinite(skin)) return fail(s, SRMD_EINVAL, "skin must be >= 0");
  const double rcm = rc_max(s);
  for (int k = 0; k < 3; ++k)
    if (!(rcm + skin < 0.5 * (double)s->Lf[k]))
      return fail(s, SRMD_EINVAL, "cutoff + skin must stay below half of every box side");
  s->skin = skin;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_integrator_nve(srmd_system *s, double dt) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(s, SRMD_EINVAL, "dt must be positive");
  s->dt = dt;
  s->thermostat = 0;
  s->integrator_set = true;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_integrator_nvt(srmd_system *s, double dt, double T0, double tau) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!(dt > 0) || !std::isfinite(dt) || !(T0 > 0) || !std::isfinite(T0) || !(tau > 0))
    return fail(s, SRMD_EINVAL, "dt, T0 and tau must be positive");
  s->dt = dt;
  s->T0 = T0;
  s->tau = tau;
  s->thermostat = 1;
  s->integrator_set = true;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_launch(srmd_system *s, int32_t tp, int32_t ppb) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (tp == 0 && ppb == 0) {
    s->tp_req = s->ppb_req = 0;
    s->dirty = true;
    return SRMD_OK;
  }
  if (tp < 1 || tp > 64 || (tp & (tp - 1)) != 0) return fail(s, SRMD_EINVAL, "tp must be a power of two in 1..64");
  if (ppb < 1 || tp * ppb > 1024 || (tp * ppb) % 64 != 0)
    return fail(s, SRMD_EINVAL, "tp * ppb must be a multiple of 64 and at most 1024");
  s->tp_req = tp;
  s->ppb_req = ppb;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_persistent(srmd_system *s, int32_t groups) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (groups < -1 || groups > 4096) return fail(s, SRMD_EINVAL, "groups must be -1, 0 or 1..4096");
  s->persist_req = groups;
  s->persist_set = true;
  int tp, ppb;
  launch_of(s, &tp, &ppb);
  if (tp != s->tp || ppb != s->ppb) {
    s->dirty = true;  // the default launch shape differs between the modes
  } else if (!s->dirty) {
    // same layout (the partials buffer always has room for the persistent kernel):
    // the list is kept and the trajectory continues
    resolve_persistent(s);
  }
  return SRMD_OK;
}

srmd_status srmd_set_rebuild_path(srmd_system *s, int32_t sort_mode, int32_t list_mode) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (sort_mode < 0 || sort_mode > 2 || list_mode < 0 || list_mode > 5)
    return fail(s, SRMD_EINVAL, "sort mode must be 0 (auto), 1 or 2 and list mode 0 (auto), 1, 2, 3 or 4");
  s->sort_mode = sort_mode;
  s->list_mode = list_mode;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_sort_interval(srmd_system *s, int32_t builds) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (builds < 0) return fail(s, SRMD_EINVAL, "the sort interval must be >= 0");
  s->sort_every = builds;
  s->dirty = true;
  return SRMD_OK;
}

srmd_status srmd_set_fused_reduction(srmd_system *s, int32_t enable) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (enable < -1 || enable > 2) return fail(s, SRMD_EINVAL, "enable must be -1, 0, 1 or 2");
  s->tail_req = enable;
  s->dirty = true;  // the captured graphs hold the other form
  return SRMD_OK;
}

srmd_status srmd_get_launch(const srmd_system *s, int32_t *tp, int32_t *ppb) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  int a, b;
  launch_of(s, &a, &b);
  if (tp) *tp = a;
  if (ppb) *ppb = b;
  return SRMD_OK;
}

srmd_status srmd_build_neighbor_list(srmd_system *s) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  for (int attempt = 0; attempt < 8; ++attempt) {
    st = request_rebuild(s);
    if (st != SRMD_OK) return st;
    st = flush_host_sort(s);
    if (st != SRMD_OK) return st;
    HIPCHK(s, launch_rebuild(s->stream, s->c, s->p, s->cur));
    st = set_ctl_int(s, offsetof(Control, rebuild), 0);
    if (st != SRMD_OK) return st;
    Control h;
    st = read_ctl(s, &h);
    if (st != SRMD_OK) return st;
    if (!(h.error & 2)) return SRMD_OK;
    st = set_ctl_int(s, offsetof(Control, error), h.error & ~2);
    if (st != SRMD_OK) return st;
    st = regrow(s);
    if (st != SRMD_OK) return st;
  }
  return fail(s, SRMD_ENOMEM, "neighbour list kept overflowing");
}

srmd_status srmd_compute_forces(srmd_system *s, srmd_thermo *out) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  for (int attempt = 0; attempt < 8; ++attempt) {
    st = flush_host_sort(s);
    if (st != SRMD_OK) return st;
    HIPCHK(s, launch_rebuild(s->stream, s->c, s->p, s->cur));
    HIPCHK(s, launch_force(s->tp, kmethod(s), step_blocks(s), s->tp * s->ppb, s->stream, s->c, s->p, s->cur));
    HIPCHK(s, launch_finish(1, step_blocks(s), s->cur, s->stream, s->c, s->p));
    Control h;
    st = read_ctl(s, &h);
    if (st != SRMD_OK) return st;
    if (h.error & 2) {
      st = set_ctl_int(s, offsetof(Control, error), h.error & ~2);
      if (st != SRMD_OK) return st;
      st = regrow(s);  // requests a rebuild
      if (st != SRMD_OK) return st;
      continue;
    }
    if (h.error & 1) return fail(s, SRMD_ESTATE, "non-finite force");
    if (out) return srmd_get_thermo(s, out);
    return SRMD_OK;
  }
  return fail(s, SRMD_ENOMEM, "neighbour list kept overflowing");
}

srmd_status srmd_step(srmd_system *s, int64_t nsteps, int32_t thermo_every, srmd_thermo *trace, int64_t trace_cap) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (nsteps < 0) return fail(s, SRMD_EINVAL, "nsteps must be >= 0");
  if (!s->integrator_set) return fail(s, SRMD_EINVAL, "integrator not set");
  if (thermo_every < 0 || trace_cap < 0 || (trace_cap > 0 && !trace))
    return fail(s, SRMD_EINVAL, "invalid trace arguments");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  if (nsteps == 0) return SRMD_OK;
  const long long cap = thermo_every > 0 ? trace_cap : 0;
  st = ensure_trace(s, cap);
  if (st != SRMD_OK) return st;
  st = alloc_snapshot(s);
  if (st != SRMD_OK) return st;
  st = run_with_replay(s, nsteps, thermo_every, cap);
  if (st != SRMD_OK) return st;
  return download_trace(s, cap, trace);
}

srmd_status srmd_get_state(srmd_system *s, float *pos, float *vel, int32_t *image, float *force, double *pos64) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  const size_t n = (size_t)s->n;
  std::vector<int4> hi(n);
  HIPCHK(s, hipMemcpyAsync(hi.data(), s->p.img, sizeof(int4) * n, hipMemcpyDeviceToHost, s->stream));
  std::vector<float4> hp(n), hv(n), hf(n);
  std::vector<double> h64;
  HIPCHK(s, hipMemcpyAsync(hp.data(), s->p.pos[s->cur], sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  if (vel) HIPCHK(s, hipMemcpyAsync(hv.data(), s->p.vel, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  if (force) HIPCHK(s, hipMemcpyAsync(hf.data(), s->p.force, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  if (pos64 && s->p.pos64) {
    h64.resize(3 * n);
    HIPCHK(s, hipMemcpyAsync(h64.data(), s->p.pos64, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (size_t k = 0; k < n; ++k) {
    const int id = hi[k].w;
    if (id < 0 || (size_t)id >= n) return fail(s, SRMD_ESTATE, "corrupt particle id on the device");
    if (pos) {
      pos[3 * id] = hp[k].x;
      pos[3 * id + 1] = hp[k].y;
      pos[3 * id + 2] = hp[k].z;
    }
    if (vel) {
      vel[3 * id] = hv[k].x;
      vel[3 * id + 1] = hv[k].y;
      vel[3 * id + 2] = hv[k].z;
    }
    if (image) {
      image[3 * id] = hi[k].x;
      image[3 * id + 1] = hi[k].y;
      image[3 * id + 2] = hi[k].z;
    }
    if (force) {
      force[3 * id] = hf[k].x;
      force[3 * id + 1] = hf[k].y;
      force[3 * id + 2] = hf[k].z;
    }
    if (pos64) {
      for (int d = 0; d < 3; ++d)
        pos64[3 * id + d] = h64.empty() ? (double)(&hp[k].x)[d] : h64[3 * k + (size_t)d];
    }
  }
  return SRMD_OK;
}

srmd_status srmd_get_particle_terms(srmd_system *s, float *pe, float *virial) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  const size_t n = (size_t)s->n;
  std::vector<int4> hi(n);
  std::vector<float4> hf(n);
  std::vector<float> hw(n);
  HIPCHK(s, hipMemcpyAsync(hi.data(), s->p.img, sizeof(int4) * n, hipMemcpyDeviceToHost, s->stream));
  if (pe) HIPCHK(s, hipMemcpyAsync(hf.data(), s->p.force, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  if (virial) HIPCHK(s, hipMemcpyAsync(hw.data(), s->p.wpart, sizeof(float) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (size_t k = 0; k < n; ++k) {
    const int id = hi[k].w;
    if (id < 0 || (size_t)id >= n) return fail(s, SRMD_ESTATE, "corrupt particle id on the device");
    if (pe) pe[id] = hf[k].w;
    if (virial) virial[id] = hw[k];
  }
  return SRMD_OK;
}

srmd_status srmd_set_state(srmd_system *s, const float *pos, const float *vel) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  const size_t n = (size_t)s->n;
  for (size_t i = 0; i < 3 * n; ++i) {
    if (pos && !std::isfinite(pos[i])) return fail(s, SRMD_EINVAL, "non-finite position");
    if (vel && !std::isfinite(vel[i])) return fail(s, SRMD_EINVAL, "non-finite velocity");
  }
  std::vector<int4> hi(n);
  std::vector<float4> hp(n);
  HIPCHK(s, hipMemcpyAsync(hi.data(), s->p.img, sizeof(int4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(hp.data(), s->p.pos[s->cur], sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  std::vector<float> P(3 * n), Vv(3 * n);
  std::vector<int32_t> T(n);
  std::vector<float> curvel;
  if (!vel) {
    std::vector<float4> hv(n);
    HIPCHK(s, hipMemcpyAsync(hv.data(), s->p.vel, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (size_t k = 0; k < n; ++k) {
      const int id = hi[k].w;
      Vv[3 * id] = hv[k].x;
      Vv[3 * id + 1] = hv[k].y;
      Vv[3 * id + 2] = hv[k].z;
    }
  }
  for (size_t k = 0; k < n; ++k) {
    const int id = hi[k].w;
    int ty;
    std::memcpy(&ty, &hp[k].w, 4);
    T[id] = ty;
    for (int d = 0; d < 3; ++d) P[3 * id + d] = pos ? pos[3 * id + d] : (&hp[k].x)[d];
    if (vel)
      for (int d = 0; d < 3; ++d) Vv[3 * id + d] = vel[3 * id + d];
  }
  srmd_status st = upload_state(s, P.data(), Vv.data(), T.data());
  if (st != SRMD_OK) return st;
  st = set_ctl_int(s, offsetof(Control, error), 0);  // errors of the replaced state do not carry over
  if (st != SRMD_OK) return st;
  return request_rebuild(s);
}

// ---------------------------------------------------------------------------
// Full-state checkpoint.  The blob holds the device state in its device (spatially
// sorted) order, so that a loaded system continues the saved trajectory bit for
// bit: positions (type bits included), velocities, images and ids, last-build
// positions, last forces, the precision residuals, the neighbour list and its
// lengths, the control block (step, rebuilds, Nose-Hoover friction and its
// integral) and the last thermodynamic record.  The list is restored only into the
// same list layout; otherwise the loaded state rebuilds it before the next force
// evaluation.

namespace {

constexpr char kStateMagic[8] = {'S', 'R', 'M', 'D', 'S', 'T', 'v', '1'};

// What a stored list depends on besides the particle order: the list geometry and
// the per-type-pair list radii.
struct ListLayout {
  int tp, n_max, nvp, ncell, nc[3], full_axis, small_sort, list_kind;
  float cs2[kMaxPairs];
};

struct StateHeader {
  char magic[8];
  int32_t n, ntypes, prec, cur_unused;
  float L[3];
  int32_t sort_state;   // 0 none pending; 1 rebuild requested, sort not yet run; 2 sort already run
  int64_t list_rows;    // rows of tp entries per particle stored (0: no list)
  ListLayout layout;
  Control ctl;
  Thermo thermo;
};

ListLayout layout_of(const srmd_system *s) {
  ListLayout l;
  std::memset(&l, 0, sizeof(l));
  l.tp = s->c.tp;
  l.n_max = s->c.n_max;
  l.nvp = s->c.nvp;
  l.ncell = s->c.ncell;
  for (int k = 0; k < 3; ++k) l.nc[k] = s->c.nc[k];
  l.full_axis = s->c.full_axis;
  l.small_sort = s->c.small_sort;
  l.list_kind = s->c.list_kind;
  for (int a = 0; a < kMaxPairs; ++a) l.cs2[a] = s->c.pt.cs2[a];
  return l;
}

size_t state_bytes(const srmd_system *s, long long rows) {
  const size_t n = (size_t)s->n;
  size_t b = sizeof(StateHeader) + n * (5 * sizeof(float4) + sizeof(int));
  if (s->p.pos64) b += 3 * n * sizeof(double);
  if (s->p.kahan) b += n * sizeof(float4);
  b += (size_t)rows * (size_t)s->c.nvp * (size_t)s->c.tp * sizeof(int);
  return b;
}

}  // namespace

srmd_status srmd_save_state(srmd_system *s, void *buf, size_t bytes, size_t *needed) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!needed) return fail(s, SRMD_EINVAL, "needed is NULL");
  srmd_status st = prepare(s);  // a pending parameter change requests its rebuild first
  if (st != SRMD_OK) return st;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  HIPCHK(s, hipMemcpyAsync(&h.ctl, s->p.ctl, sizeof(Control), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(&h.thermo, s->p.thermo, sizeof(Thermo), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  // the list is stored when it is the one the next force evaluation uses
  const long long rows = h.ctl.rebuild ? 0 : (h.ctl.max_nbrs + s->c.tp - 1) / s->c.tp;
  *needed = state_bytes(s, rows);
  if (!buf) return SRMD_OK;
  if (bytes < *needed) return fail(s, SRMD_EINVAL, "state buffer too small");
  std::memcpy(h.magic, kStateMagic, 8);
  h.n = s->n;
  h.ntypes = s->ntypes;
  h.prec = (int32_t)s->prec;
  for (int k = 0; k < 3; ++k) h.L[k] = s->Lf[k];
  h.sort_state = !h.ctl.rebuild ? 0 : (s->c.small_sort && !s->sort_pending) ? 2 : 1;
  h.list_rows = rows;
  h.layout = layout_of(s);
  const size_t n = (size_t)s->n;
  char *q = (char *)buf;
  std::memcpy(q, &h, sizeof(h));
  q += sizeof(h);
  auto d2h = [&](const void *src, size_t b) {
    hipError_t e = hipMemcpyAsync(q, src, b, hipMemcpyDeviceToHost, s->stream);
    q += b;
    return e;
  };
  HIPCHK(s, d2h(s->p.pos[s->cur], sizeof(float4) * n));
  HIPCHK(s, d2h(s->p.vel, sizeof(float4) * n));
  HIPCHK(s, d2h(s->p.img, sizeof(int4) * n));
  HIPCHK(s, d2h(s->p.last, sizeof(float4) * n));
  HIPCHK(s, d2h(s->p.force, sizeof(float4) * n));
  HIPCHK(s, d2h(s->p.nnb, sizeof(int) * n));
  if (s->p.pos64) HIPCHK(s, d2h(s->p.pos64, 3 * sizeof(double) * n));
  if (s->p.kahan) HIPCHK(s, d2h(s->p.kahan, sizeof(float4) * n));
  if (rows > 0) HIPCHK(s, d2h(s->p.nbl, (size_t)rows * (size_t)s->c.nvp * (size_t)s->c.tp * sizeof(int)));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

srmd_status srmd_load_state(srmd_system *s, const void *buf, size_t bytes) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!buf || bytes < sizeof(StateHeader)) return fail(s, SRMD_EINVAL, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(s, SRMD_EINVAL, "not a saved srmd state");
  if (h.n != s->n || h.ntypes != s->ntypes || h.prec != (int32_t)s->prec)
    return fail(s, SRMD_EINVAL, "saved state has another particle count, type count or precision");
  for (int k = 0; k < 3; ++k)
    if (h.L[k] != s->Lf[k]) return fail(s, SRMD_EINVAL, "saved state has another box");
  if (h.list_rows < 0 || h.list_rows > h.layout.n_max || h.layout.tp < 1 || h.layout.nvp < h.n)
    return fail(s, SRMD_EINVAL, "corrupt saved state header");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  const size_t n = (size_t)s->n;
  size_t need = sizeof(StateHeader) + n * (5 * sizeof(float4) + sizeof(int));
  if (s->p.pos64) need += 3 * n * sizeof(double);
  if (s->p.kahan) need += n * sizeof(float4);
  const size_t list_b = (size_t)h.list_rows * (size_t)h.layout.nvp * (size_t)h.layout.tp * sizeof(int);
  if (bytes != need + list_b) return fail(s, SRMD_EINVAL, "state buffer size does not match its header");
  // every particle id appears once and every type is in range
  const char *q = (const char *)buf + sizeof(StateHeader);
  {
    const float4 *hp = (const float4 *)q;
    const int4 *hi = (const int4 *)(q + 2 * sizeof(float4) * n);
    std::vector<char> seen(n, 0);
    for (size_t k = 0; k < n; ++k) {
      int ty;
      std::memcpy(&ty, &hp[k].w, 4);
      const int id = hi[k].w;
      if (ty < 0 || ty >= s->ntypes || id < 0 || (size_t)id >= n || seen[(size_t)id])
        return fail(s, SRMD_EINVAL, "corrupt saved state (types or particle ids)");
      seen[(size_t)id] = 1;
    }
  }
  const ListLayout cur = layout_of(s);
  const bool keep_list = std::memcmp(&cur, &h.layout, sizeof(ListLayout)) == 0 && h.sort_state == 0;
  auto h2d = [&](void *dst, size_t b) {
    hipError_t e = hipMemcpyAsync(dst, q, b, hipMemcpyHostToDevice, s->stream);
    q += b;
    return e;
  };
  HIPCHK(s, h2d(s->p.pos[s->cur], sizeof(float4) * n));
  HIPCHK(s, h2d(s->p.vel, sizeof(float4) * n));
  HIPCHK(s, h2d(s->p.img, sizeof(int4) * n));
  HIPCHK(s, h2d(s->p.last, sizeof(float4) * n));
  HIPCHK(s, h2d(s->p.force, sizeof(float4) * n));
  if (keep_list) {
    HIPCHK(s, h2d(s->p.nnb, sizeof(int) * n));
  } else {
    q += sizeof(int) * n;
  }
  if (s->p.pos64) HIPCHK(s, h2d(s->p.pos64, 3 * sizeof(double) * n));
  if (s->p.kahan) HIPCHK(s, h2d(s->p.kahan, sizeof(float4) * n));
  if (keep_list) HIPCHK(s, h2d(s->p.nbl, list_b));
  Control c = h.ctl;
  c.error = 0;
  if (!keep_list) {
    // the list is rebuilt (spatial sort first) before the next force evaluation; a
    // sort the saved run already performed counts its rebuild once
    if (h.sort_state == 2) c.n_rebuilds -= 1;
    c.rebuild = 1;
    s->sort_pending = true;
  } else {
    s->sort_pending = false;
  }
  HIPCHK(s, hipMemcpyAsync(s->p.ctl, &c, sizeof(Control), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->p.thermo, &h.thermo, sizeof(Thermo), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return SRMD_OK;
}

srmd_status srmd_get_neighbor_pairs(srmd_system *s, int32_t *pairs, int64_t cap, int64_t *count) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!count) return fail(s, SRMD_EINVAL, "count is NULL");
  if (!s->p.nbl) return fail(s, SRMD_EINVAL, "no neighbour list has been built");
  const size_t n = (size_t)s->n;
  std::vector<int4> hi(n);
  std::vector<int> nn(n);
  std::vector<int> nb((size_t)s->c.n_max * (size_t)s->c.nvp);
  HIPCHK(s, hipMemcpyAsync(hi.data(), s->p.img, sizeof(int4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(nn.data(), s->p.nnb, sizeof(int) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(nb.data(), s->p.nbl, sizeof(int) * nb.size(), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  long long total = 0;
  for (size_t t = 0; t < n; ++t) total += nn[t];
  *count = total;
  if (!pairs) return SRMD_OK;
  if (total > cap) return fail(s, SRMD_EINVAL, "pair buffer too small");
  std::vector<std::pair<int, int>> v;
  v.reserve((size_t)total);
  const long long tp = s->c.tp, nvp = s->c.nvp;
  for (size_t t = 0; t < n; ++t) {
    for (int k = 0; k < nn[t]; ++k) {
      const long long addr = (long long)(k / tp) * (nvp * tp) + (long long)t * tp + (k % tp);
      const int u = nb[(size_t)addr];
      if (u < 0 || (size_t)u >= n) return fail(s, SRMD_ESTATE, "corrupt neighbour index");
      v.emplace_back(hi[t].w, hi[(size_t)u].w);
    }
  }
  std::sort(v.begin(), v.end());
  for (size_t k = 0; k < v.size(); ++k) {
    pairs[2 * k] = v[k].first;
    pairs[2 * k + 1] = v[k].second;
  }
  return SRMD_OK;
}

srmd_status srmd_get_thermo(srmd_system *s, srmd_thermo *out) {
  if (!s || !out) return fail(s, SRMD_EINVAL, "NULL argument");
  Thermo t;
  HIPCHK(s, hipMemcpyAsync(&t, s->p.thermo, sizeof(Thermo), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  to_public(t, out);
  return SRMD_OK;
}

srmd_status srmd_get_box(const srmd_system *s, double box[3]) {
  if (!s || !box) return fail(nullptr, SRMD_EINVAL, "NULL argument");
  for (int k = 0; k < 3; ++k) box[k] = (double)s->Lf[k];
  return SRMD_OK;
}

srmd_status srmd_get_stats(srmd_system *s, srmd_stats *out) {
  if (!s || !out) return fail(s, SRMD_EINVAL, "NULL argument");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  Control h;
  st = read_ctl(s, &h);
  if (st != SRMD_OK) return st;
  out->steps = h.step;
  out->n_rebuilds = h.n_rebuilds;
  out->list_entries = h.list_entries;
  out->max_nbrs = h.max_nbrs;
  out->n_max = s->c.n_max;
  out->tp = s->tp;
  out->ppb = s->ppb;
  out->blocks = step_blocks(s);
  out->ncell = s->c.ncell;
  out->persistent_groups = s->persist_groups;
  out->list_mode = s->c.list_kind;
  out->step_form = s->persist_groups > 0 ? 0 : step_tail(s);
  out->reserved = 0;
  return SRMD_OK;
}

srmd_status srmd_profile_step_kernel(srmd_system *s, int64_t nsteps, double *kernel_ms, double *device_ms,
                                     int64_t *launches) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (nsteps < 0) return fail(s, SRMD_EINVAL, "nsteps must be >= 0");
  if (!s->integrator_set) return fail(s, SRMD_EINVAL, "integrator not set");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  Control h;
  st = read_ctl(s, &h);
  if (st != SRMD_OK) return st;
  h.prof_ticks = 0;
  h.prof_count = 0;
  h.thermo_every = 0;
  h.trace_cap = 0;
  st = h2d_sync(s, s->p.ctl, &h, sizeof(Control));
  if (st != SRMD_OK) return st;
  const int batch = 256;  // events per synchronisation
  std::vector<hipEvent_t> ev(2 * batch);
  for (auto &e : ev) HIPCHK(s, hipEventCreate(&e));
  double total = 0.0;
  long long done = 0;
  srmd_status result = SRMD_OK;
  st = flush_host_sort(s);
  if (st != SRMD_OK) result = st;
  if (result == SRMD_OK && !s->persist_err.empty()) result = fail(s, SRMD_EUNSUPPORTED, s->persist_err);
  if (result == SRMD_OK && s->persist_groups > 0) {
    // persistent mode: one event pair around each launch of kPersistChunk steps, all
    // enqueued back to back (the launches run as in srmd_step), read at the end
    const long long nl = (nsteps + kPersistChunk - 1) / kPersistChunk;
    for (long long k = (long long)ev.size(); k < 2 * nl && result == SRMD_OK; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) result = fail(s, SRMD_EHIP, "hipEventCreate failed");
      else ev.push_back(e);
    }
    for (long long k = 0; k < nl && result == SRMD_OK; ++k) {
      const int cnt = (int)std::min<long long>(kPersistChunk, nsteps - done);
      hipError_t e = hipEventRecord(ev[2 * k], s->stream);
      if (e == hipSuccess) {
        result = launch_persistent(s, cnt);
        if (result == SRMD_OK) e = hipEventRecord(ev[2 * k + 1], s->stream);
      }
      if (e != hipSuccess && result == SRMD_OK)
        result = fail(s, SRMD_EHIP, std::string("persistent profiled launch: ") + hipGetErrorString(e));
      done += cnt;
    }
    if (result == SRMD_OK && nl > 0) {
      hipError_t e = hipEventSynchronize(ev[2 * nl - 1]);
      for (long long k = 0; k < nl && e == hipSuccess; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
        total += ms;
      }
      if (e != hipSuccess) result = fail(s, SRMD_EHIP, std::string("persistent profile events: ") + hipGetErrorString(e));
    }
    for (auto &ev_k : ev) (void)hipEventDestroy(ev_k);
    if (result != SRMD_OK) return result;
    st = read_ctl(s, &h);
    if (st != SRMD_OK) return st;
    st = check_barrier(s, &h);
    if (st != SRMD_OK) return st;
    if (h.error & 3) return fail(s, SRMD_ESTATE, "list overflow or non-finite state during profiling");
    if (kernel_ms) *kernel_ms = total;
    if (device_ms) *device_ms = 0.0;
    if (launches) *launches = nl;
    return SRMD_OK;
  }
  while (done < nsteps && result == SRMD_OK) {
    const int cnt = (int)std::min<long long>(batch, nsteps - done);
    for (int k = 0; k < cnt && result == SRMD_OK; ++k) {
      const int tail = step_tail(s);
      hipError_t e = tail == 2 ? hipSuccess : launch_rebuild(s->stream, s->c, s->p, s->cur);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * k], s->stream);
      if (e == hipSuccess)
        e = launch_step(s->tp, kmethod(s), (int)s->prec, step_blocks(s), s->tp * s->ppb, s->stream, s->c, s->p, s->cur,
                        tail, tail ? tail_lds_bytes(s->c, s->tp * s->ppb, tail) : 0);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * k + 1], s->stream);
      if (e == hipSuccess && !tail) e = launch_finish(0, step_blocks(s), s->cur ^ 1, s->stream, s->c, s->p);
      if (e != hipSuccess) result = fail(s, SRMD_EHIP, std::string("profiled launch: ") + hipGetErrorString(e));
      s->cur ^= 1;
    }
    if (result != SRMD_OK) break;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
      result = fail(s, SRMD_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
      break;
    }
    for (int k = 0; k < cnt; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
      if (e != hipSuccess) {
        result = fail(s, SRMD_EHIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
        break;
      }
      total += ms;
    }
    done += cnt;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (result != SRMD_OK) return result;
  st = read_ctl(s, &h);
  if (st != SRMD_OK) return st;
  if (h.error & 3) return fail(s, SRMD_ESTATE, "list overflow or non-finite state during profiling");
  int rate_khz = 0;
  HIPCHK(s, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0));
  if (kernel_ms) *kernel_ms = total;
  if (device_ms) *device_ms = rate_khz > 0 ? (double)h.prof_ticks / (double)rate_khz : 0.0;
  if (launches) *launches = done;
  return SRMD_OK;
}

srmd_status srmd_autotune(srmd_system *s, int32_t steps_per_trial, int32_t *tp_out, int32_t *ppb_out) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!s->integrator_set) return fail(s, SRMD_EINVAL, "integrator not set");
  if (steps_per_trial < 1) return fail(s, SRMD_EINVAL, "steps_per_trial must be >= 1");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  HostState saved;
  st = save_host_state(s, &saved);
  if (st != SRMD_OK) return st;
  const int tp0 = s->tp_req, ppb0 = s->ppb_req, list0 = s->list_mode;
  const int preq0 = s->persist_req;
  const bool pset0 = s->persist_set;
  hipEvent_t e0, e1;
  HIPCHK(s, hipEventCreate(&e0));
  HIPCHK(s, hipEventCreate(&e1));
  // one timed trial from the stored state (paper appendix: every run starts from the same configuration)
  auto trial = [&](int tp, int ppb, int list_mode, bool persistent, double *ms_per_step) -> srmd_status {
    s->tp_req = tp;
    s->ppb_req = ppb;
    s->list_mode = list_mode;
    s->persist_set = true;
    s->persist_req = persistent ? -1 : 0;
    s->dirty = true;
    srmd_status r = restore_host_state(s, saved);
    if (r != SRMD_OK) return r;
    r = prepare(s);
    if (r != SRMD_OK) return r;
    if (persistent && s->persist_groups == 0) {  // not available for this system
      *ms_per_step = 1e30;
      return SRMD_OK;
    }
    r = run_steps(s, 16);  // graph instantiation and the first build, untimed
    if (r != SRMD_OK) return r;
    HIPCHK(s, hipEventRecord(e0, s->stream));
    r = run_steps(s, steps_per_trial);
    if (r != SRMD_OK) return r;
    HIPCHK(s, hipEventRecord(e1, s->stream));
    HIPCHK(s, hipEventSynchronize(e1));
    Control h;
    r = read_ctl(s, &h);
    if (r != SRMD_OK) return r;
    r = check_barrier(s, &h);
    if (r != SRMD_OK) return r;
    float ms = 0.f;
    HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
    // a trial that overflowed its list or went non-finite does not count
    *ms_per_step = (h.error & 3) ? 1e30 : (double)ms / steps_per_trial;
    if (h.error & 3) {
      h.error &= ~3;
      r = h2d_sync(s, s->p.ctl, &h, sizeof(Control));
    }
    return r;
  };
  const int n = s->n;
  int best_tp = 0, best_ppb = 0, best_list = 0;
  double best = 1e300;
  srmd_status result = SRMD_OK;
  // Phase I: the list-build method at the default layout (paper appendix, step 3)
  int dtp, dppb;
  s->tp_req = s->ppb_req = 0;
  launch_of(s, &dtp, &dppb);
  double phase1[6] = {1e300, 1e300, 1e300, 1e300, 1e300, 1e300};
  for (int lm = 1; lm <= 5 && result == SRMD_OK; ++lm) {
    if (lm == 4 && !s->c.small_sort) continue;  // all pairs: small systems only
    double t;
    result = trial(dtp, dppb, lm, false, &t);
    if (result != SRMD_OK) break;
    phase1[lm] = t;
    if (t < best) {
      best = t;
      best_tp = dtp;
      best_ppb = dppb;
      best_list = lm;
    }
  }
  // Phase II: block size x threads per particle (paper appendix, step 4), with its stop
  // rules: leave the t_p loop after 3 slower trials in a row or one more than 5% slower,
  // and the block loop once a block size ends more than 10% slower than the best.  It
  // runs for every list method within kTunerListKeep of the fastest at the default
  // layout, as two methods that close can change places at another layout.
  const int blocks[] = {64, 128, 256, 512, 1024};
  const int tp_max = n > 100000 ? 2 : 64;  // size pruning: large systems only need t_p = 1, 2
  const double phase1_best = best;
  for (int lm = 1; lm <= 5 && result == SRMD_OK; ++lm) {
    if (!(phase1[lm] <= kTunerListKeep * phase1_best)) continue;
    double prev_block_best = 1e300;
    for (int bi = 0; bi < 5 && result == SRMD_OK; ++bi) {
      const int bsz = blocks[bi];
      double block_best = 1e300;
      int slower = 0;
      for (int tp = 1; tp <= tp_max && tp <= bsz && result == SRMD_OK; tp <<= 1) {
        double t;
        result = trial(tp, bsz / tp, lm, false, &t);
        if (result != SRMD_OK) break;
        if (t < block_best) {
          block_best = t;
          slower = 0;
        } else {
          ++slower;
        }
        if (t < best) {
          best = t;
          best_tp = tp;
          best_ppb = bsz / tp;
          best_list = lm;
        }
        if (slower >= 3 || t > 1.05 * block_best) break;
      }
      if (block_best > 1.10 * std::min(best, prev_block_best) && bi > 0) break;
      prev_block_best = std::min(prev_block_best, block_best);
    }
  }
  // Phase III (MI355X): the persistent kernel, t_p at 256-thread virtual blocks,
  // with the t_p stop rule of phase II (tp values it cannot run end the phase)
  bool best_persist = false;
  if (result == SRMD_OK && s->prec == SRMD_PREC_F32) {
    double pbest = 1e300;
    int slower = 0;
    for (int tp = 1; tp <= 64 && result == SRMD_OK; tp <<= 1) {
      double t;
      result = trial(tp, 256 / tp, best_list, true, &t);
      if (result != SRMD_OK) break;
      if (t >= 1e30) break;
      if (t < pbest) {
        pbest = t;
        slower = 0;
      } else {
        ++slower;
      }
      if (t < best) {
        best = t;
        best_tp = tp;
        best_ppb = 256 / tp;
        best_persist = true;
      }
      if (slower >= 3 || t > 1.05 * pbest) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // keep the user's explicit layout request if there was one; otherwise use the tuned one
  s->tp_req = tp0;
  s->ppb_req = ppb0;
  s->list_mode = list0;
  s->persist_req = preq0;
  s->persist_set = pset0;
  if (result == SRMD_OK && best_tp > 0) {
    s->tp_tuned = best_tp;
    s->ppb_tuned = best_ppb;
    s->persist_tuned = best_persist ? -1 : 0;
    if (list0 == 0) s->list_mode = best_list;
  }
  s->dirty = true;
  srmd_status r2 = restore_host_state(s, saved);
  if (result == SRMD_OK) result = r2;
  if (result == SRMD_OK) result = prepare(s);
  if (result != SRMD_OK) return result;
  if (tp_out) *tp_out = best_tp;
  if (ppb_out) *ppb_out = best_ppb;
  return SRMD_OK;
}

// ---------------------------------------------------------------------------
// Tuned-parameter file (paper appendix, step 8).  One text line per record:
//   srmd-tuning-v3 gpu=<name> cus=<n> prec=<p> method=<m> thermostat=<t> ntypes=<k>
//   count=<c_0,...> dt=<x> temperature=<x> density=<x> sigma=<k*k values>
//   epsilon=<k*k values> rcut=<k*k values> potential=<n> param=<4*k*k values>
//   charge=<k values> rcc=<x> tp=<n> ppb=<n> list=<n> persistent=<n> skin=<x> sort=<n>
// (records of another version are skipped)
// Floating-point fields are printed with 17 significant digits, so they read back
// to the same double.
}  // extern "C"

namespace {

constexpr const char *kTuneTag = "srmd-tuning-v3";
constexpr double kTuneRelTol = 1e-6;   // dt, density and pair parameters
constexpr double kTuneTempTol = 0.02;  // temperature

std::string gpu_token(const char *g) {
  std::string r;
  for (size_t i = 0; i < sizeof(srmd_tuning_key::gpu) && g[i]; ++i)
    r += (std::isspace((unsigned char)g[i]) || g[i] == '=' || g[i] == ',') ? '_' : g[i];
  return r.empty() ? std::string("unknown") : r;
}

bool rel_close(double a, double b, double tol) { return std::fabs(a - b) <= tol * std::max(std::fabs(a), std::fabs(b)); }

bool key_valid(const srmd_tuning_key &k) { return k.ntypes >= 1 && k.ntypes <= kMaxTypes; }

bool tuning_valid(const srmd_tuning &t) {
  const bool tp_ok = t.tp >= 1 && t.tp <= 64 && (t.tp & (t.tp - 1)) == 0;
  const bool ppb_ok = t.ppb >= 1 && (long long)t.tp * t.ppb <= 1024 && (t.tp * t.ppb) % 64 == 0;
  return tp_ok && ppb_ok && t.list_mode >= 1 && t.list_mode <= 5 && (t.persistent == 0 || t.persistent == -1) &&
         t.skin >= 0 && std::isfinite(t.skin) && t.sort_every >= 0;
}

bool key_match(const srmd_tuning_key &a, const srmd_tuning_key &b) {
  if (gpu_token(a.gpu) != gpu_token(b.gpu) || a.compute_units != b.compute_units || a.precision != b.precision ||
      a.cutoff_method != b.cutoff_method || a.thermostat != b.thermostat || a.ntypes != b.ntypes)
    return false;
  for (int t = 0; t < a.ntypes; ++t)
    if (a.count[t] != b.count[t]) return false;
  if (!rel_close(a.dt, b.dt, kTuneRelTol) || !rel_close(a.density, b.density, kTuneRelTol) ||
      !rel_close(a.temperature, b.temperature, kTuneTempTol))
    return false;
  for (int q = 0; q < a.ntypes * a.ntypes; ++q) {
    if (!rel_close(a.sigma[q], b.sigma[q], kTuneRelTol) || !rel_close(a.epsilon[q], b.epsilon[q], kTuneRelTol) ||
        !rel_close(a.rcut[q], b.rcut[q], kTuneRelTol))
      return false;
    for (int r = 0; r < 4; ++r)
      if (!rel_close(a.pot_param[q][r], b.pot_param[q][r], kTuneRelTol)) return false;
  }
  if (a.potential != b.potential || !rel_close(a.rc_coulomb, b.rc_coulomb, kTuneRelTol)) return false;
  for (int t = 0; t < a.ntypes; ++t)
    if (!rel_close(a.charge[t], b.charge[t], kTuneRelTol)) return false;
  return true;
}

std::string tuning_line(const srmd_tuning_key &k, const srmd_tuning &t) {
  std::string o = kTuneTag;
  char buf[64];
  auto num = [&](double x) {
    std::snprintf(buf, sizeof buf, "%.17g", x);
    return std::string(buf);
  };
  auto field = [&](const char *name, const std::string &v) {
    o += ' ';
    o += name;
    o += '=';
    o += v;
  };
  auto nums = [&](const double *v, int m) {
    std::string r;
    for (int q = 0; q < m; ++q) r += (q ? "," : "") + num(v[q]);
    return r;
  };
  field("gpu", gpu_token(k.gpu));
  field("cus", std::to_string(k.compute_units));
  field("prec", std::to_string(k.precision));
  field("method", std::to_string(k.cutoff_method));
  field("thermostat", std::to_string(k.thermostat));
  field("ntypes", std::to_string(k.ntypes));
  std::string cnt;
  for (int q = 0; q < k.ntypes; ++q) cnt += (q ? "," : "") + std::to_string((long long)k.count[q]);
  field("count", cnt);
  field("dt", num(k.dt));
  field("temperature", num(k.temperature));
  field("density", num(k.density));
  field("sigma", nums(k.sigma, k.ntypes * k.ntypes));
  field("epsilon", nums(k.epsilon, k.ntypes * k.ntypes));
  field("rcut", nums(k.rcut, k.ntypes * k.ntypes));
  field("potential", std::to_string(k.potential));
  field("param", nums(&k.pot_param[0][0], 4 * k.ntypes * k.ntypes));
  field("charge", nums(k.charge, k.ntypes));
  field("rcc", num(k.rc_coulomb));
  field("tp", std::to_string(t.tp));
  field("ppb", std::to_string(t.ppb));
  field("list", std::to_string(t.list_mode));
  field("persistent", std::to_string(t.persistent));
  field("skin", num(t.skin));
  field("sort", std::to_string(t.sort_every));
  return o;
}

// Split "a,b,c" and parse exactly m numbers (integers when ints is set).
bool parse_list(const std::string &s, int m, double *d, long long *ll) {
  size_t pos = 0;
  for (int q = 0; q < m; ++q) {
    const size_t end = s.find(',', pos);
    const std::string tok = s.substr(pos, end == std::string::npos ? std::string::npos : end - pos);
    if (tok.empty()) return false;
    char *e = nullptr;
    if (ll) {
      ll[q] = std::strtoll(tok.c_str(), &e, 10);
    } else {
      d[q] = std::strtod(tok.c_str(), &e);
      if (!std::isfinite(d[q])) return false;
    }
    if (!e || *e != '\0') return false;
    if ((end == std::string::npos) != (q == m - 1)) return false;
    pos = end + 1;
  }
  return true;
}

bool parse_tuning_line(const std::string &line, srmd_tuning_key *k, srmd_tuning *t) {
  std::map<std::string, std::string> kv;
  size_t pos = 0;
  bool first = true;
  while (pos < line.size()) {
    while (pos < line.size() && std::isspace((unsigned char)line[pos])) ++pos;
    if (pos >= line.size()) break;
    size_t end = pos;
    while (end < line.size() && !std::isspace((unsigned char)line[end])) ++end;
    const std::string tok = line.substr(pos, end - pos);
    pos = end;
    if (first) {
      if (tok != kTuneTag) return false;
      first = false;
      continue;
    }
    const size_t eq = tok.find('=');
    if (eq == std::string::npos || eq == 0) return false;
    kv[tok.substr(0, eq)] = tok.substr(eq + 1);
  }
  if (first) return false;
  auto one_int = [&](const char *name, long long *v) {
    auto it = kv.find(name);
    return it != kv.end() && parse_list(it->second, 1, nullptr, v);
  };
  auto one_num = [&](const char *name, double *v) {
    auto it = kv.find(name);
    return it != kv.end() && parse_list(it->second, 1, v, nullptr);
  };
  std::memset(k, 0, sizeof(*k));
  std::memset(t, 0, sizeof(*t));
  long long v[8];
  auto gi = kv.find("gpu");
  if (gi == kv.end() || gi->second.empty() || gi->second.size() >= sizeof(k->gpu)) return false;
  std::memcpy(k->gpu, gi->second.c_str(), gi->second.size());
  if (!one_int("cus", &v[0]) || !one_int("prec", &v[1]) || !one_int("method", &v[2]) ||
      !one_int("thermostat", &v[3]) || !one_int("ntypes", &v[4]))
    return false;
  if (v[4] < 1 || v[4] > kMaxTypes) return false;
  k->compute_units = (int32_t)v[0];
  k->precision = (int32_t)v[1];
  k->cutoff_method = (int32_t)v[2];
  k->thermostat = (int32_t)v[3];
  k->ntypes = (int32_t)v[4];
  const int nt = k->ntypes;
  long long cnt[kMaxTypes];
  auto ci = kv.find("count");
  if (ci == kv.end() || !parse_list(ci->second, nt, nullptr, cnt)) return false;
  for (int q = 0; q < nt; ++q) k->count[q] = cnt[q];
  if (!one_num("dt", &k->dt) || !one_num("temperature", &k->temperature) || !one_num("density", &k->density))
    return false;
  const char *arr_names[3] = {"sigma", "epsilon", "rcut"};
  double *arrs[3] = {k->sigma, k->epsilon, k->rcut};
  for (int a = 0; a < 3; ++a) {
    auto it = kv.find(arr_names[a]);
    if (it == kv.end() || !parse_list(it->second, nt * nt, arrs[a], nullptr)) return false;
  }
  {
    auto pi = kv.find("param"), qi = kv.find("charge");
    if (!one_int("potential", &v[0]) || v[0] < 0 || v[0] > 6 || pi == kv.end() || qi == kv.end() ||
        !parse_list(pi->second, 4 * nt * nt, &k->pot_param[0][0], nullptr) ||
        !parse_list(qi->second, nt, k->charge, nullptr) || !one_num("rcc", &k->rc_coulomb))
      return false;
    k->potential = (int32_t)v[0];
  }
  if (!one_int("tp", &v[0]) || !one_int("ppb", &v[1]) || !one_int("list", &v[2]) || !one_int("persistent", &v[3]) ||
      !one_num("skin", &t->skin) || !one_int("sort", &v[4]) || v[4] < 0 || v[4] > (1 << 20))
    return false;
  t->sort_every = (int32_t)v[4];
  for (int q = 0; q < 4; ++q)
    if (v[q] < -1 || v[q] > 1024) return false;
  t->tp = (int32_t)v[0];
  t->ppb = (int32_t)v[1];
  t->list_mode = (int32_t)v[2];
  t->persistent = (int32_t)v[3];
  return tuning_valid(*t);
}

}  // namespace

extern "C" {

srmd_status srmd_tuning_cache_find(const char *path, const srmd_tuning_key *key, srmd_tuning *out, int32_t *found) {
  if (!path || !key || !out || !found) return fail(nullptr, SRMD_EINVAL, "path, key, out and found are required");
  if (!key_valid(*key)) return fail(nullptr, SRMD_EINVAL, "key.ntypes must be in 1..4");
  *found = 0;
  FILE *f = std::fopen(path, "r");
  if (!f) return SRMD_OK;  // no file: nothing tuned yet
  std::string line;
  char buf[1024];
  srmd_tuning best{};
  while (std::fgets(buf, sizeof buf, f)) {
    line += buf;
    if (line.empty() || line.back() != '\n') {
      if (!std::feof(f)) continue;  // a line longer than the buffer: keep reading it
    }
    srmd_tuning_key k;
    srmd_tuning t;
    if (parse_tuning_line(line, &k, &t) && key_match(*key, k)) {
      best = t;
      *found = 1;
    }
    line.clear();
  }
  std::fclose(f);
  if (*found) {
    best.from_cache = 1;
    *out = best;
  }
  return SRMD_OK;
}

srmd_status srmd_tuning_cache_store(const char *path, const srmd_tuning_key *key, const srmd_tuning *t) {
  if (!path || !key || !t) return fail(nullptr, SRMD_EINVAL, "path, key and tuning are required");
  if (!key_valid(*key)) return fail(nullptr, SRMD_EINVAL, "key.ntypes must be in 1..4");
  if (!tuning_valid(*t)) return fail(nullptr, SRMD_EINVAL, "tuning values out of range");
  FILE *f = std::fopen(path, "a");
  if (!f) return fail(nullptr, SRMD_EINVAL, std::string("cannot open ") + path + " for appending");
  const std::string line = tuning_line(*key, *t) + "\n";
  const bool ok = std::fwrite(line.data(), 1, line.size(), f) == line.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed) return fail(nullptr, SRMD_EINVAL, std::string("write to ") + path + " failed");
  return SRMD_OK;
}

srmd_status srmd_tuning_key_of(srmd_system *s, srmd_tuning_key *key) {
  if (!s || !key) return fail(s, SRMD_EINVAL, "system and key are required");
  if (!s->integrator_set) return fail(s, SRMD_EINVAL, "integrator not set");
  if (s->method < 0 || !all_pairs_given(s))
    return fail(s, SRMD_EINVAL, "pair potential not set for every type pair (srmd_set_pair_lj)");
  std::memset(key, 0, sizeof(*key));
  int dev = 0;
  HIPCHK(s, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(s, hipGetDeviceProperties(&prop, dev));
  const std::string g = gpu_token(prop.gcnArchName);
  std::memcpy(key->gpu, g.c_str(), std::min(g.size(), sizeof(key->gpu) - 1));
  key->compute_units = prop.multiProcessorCount;
  key->precision = (int32_t)s->prec;
  key->cutoff_method = kmethod(s);
  key->thermostat = s->thermostat;
  key->ntypes = s->ntypes;
  const size_t n = (size_t)s->n;
  std::vector<float4> pos(n), vel(n);
  HIPCHK(s, hipMemcpyAsync(pos.data(), s->p.pos[s->cur], sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(vel.data(), s->p.vel, sizeof(float4) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  double ke = 0.0;
  for (size_t i = 0; i < n; ++i) {
    int ty;
    std::memcpy(&ty, &pos[i].w, 4);  // the type travels in the fourth component
    if (ty < 0 || ty >= s->ntypes) return fail(s, SRMD_ESTATE, "particle type out of range on the device");
    key->count[ty] += 1;
    const double vx = vel[i].x, vy = vel[i].y, vz = vel[i].z;
    ke += 0.5 * s->mass[ty] * (vx * vx + vy * vy + vz * vz);
  }
  key->density = (double)s->n / ((double)s->Lf[0] * (double)s->Lf[1] * (double)s->Lf[2]);
  key->temperature = s->thermostat ? s->T0 : 2.0 * ke / (3.0 * (double)s->n - 3.0);
  key->dt = s->dt;
  for (int a = 0; a < s->ntypes; ++a)
    for (int b = 0; b < s->ntypes; ++b) {
      const int q = a * s->ntypes + b, pi = pair_index(s, a, b);
      key->sigma[q] = s->sigma[pi];
      key->epsilon[q] = s->eps[pi];
      key->rcut[q] = s->rc[pi];
      if (s->pot == 1) {
        key->pot_param[q][0] = s->mie_a[pi];
        key->pot_param[q][1] = s->mie_b[pi];
        key->pot_param[q][2] = s->mie_m[pi];
        key->pot_param[q][3] = s->mie_n[pi];
      } else if (s->pot >= 2) {
        for (int r = 0; r < 4; ++r) key->pot_param[q][r] = s->gen_p[pi][r];
      }
    }
  key->potential = s->pot >= 1 ? s->pot : 0;
  if (s->coulomb) {
    for (int t = 0; t < s->ntypes; ++t) key->charge[t] = s->charge[t];
    key->rc_coulomb = s->rcc;
  }
  return SRMD_OK;
}

}  // extern "C"

namespace {

// Make t the system's settings, as the explicit setters would.
void apply_tuning(srmd_system *s, const srmd_tuning &t) {
  s->tp_req = t.tp;
  s->ppb_req = t.ppb;
  s->list_mode = t.list_mode;
  s->persist_req = t.persistent;
  s->persist_set = true;
  s->skin = t.skin;
  s->sort_every = t.sort_every;
  s->dirty = true;
}

bool skin_fits(const srmd_system *s, double skin) {
  if (!(skin > 0) || !std::isfinite(skin)) return false;
  const double rcm = rc_max(s);
  for (int k = 0; k < 3; ++k)
    if (!(rcm + skin < 0.5 * (double)s->Lf[k])) return false;
  return true;
}

}  // namespace

extern "C" {

srmd_status srmd_autotune_full(srmd_system *s, int32_t steps_per_trial, const char *cache_path, srmd_tuning *out) {
  if (!s) return fail(nullptr, SRMD_EINVAL, "system is NULL");
  if (!s->integrator_set) return fail(s, SRMD_EINVAL, "integrator not set");
  if (steps_per_trial < 1) return fail(s, SRMD_EINVAL, "steps_per_trial must be >= 1");
  srmd_status st = prepare(s);
  if (st != SRMD_OK) return st;
  srmd_tuning_key key{};
  if (cache_path) {
    st = srmd_tuning_key_of(s, &key);
    if (st != SRMD_OK) return st;
    srmd_tuning hit{};
    int32_t found = 0;
    st = srmd_tuning_cache_find(cache_path, &key, &hit, &found);
    if (st != SRMD_OK) return fail(s, st, srmd_last_error(nullptr));
    if (found && skin_fits(s, hit.skin)) {
      // a record from the same user parameters: applied without timing anything
      const int tp0 = s->tp_req, ppb0 = s->ppb_req, lm0 = s->list_mode, pr0 = s->persist_req;
      const bool ps0 = s->persist_set;
      const double sk0 = s->skin;
      apply_tuning(s, hit);
      st = prepare(s);
      if (st == SRMD_OK && s->persist_err.empty()) {
        if (out) *out = hit;
        return SRMD_OK;
      }
      // the record does not fit this system after all (e.g. another box shape): tune
      s->tp_req = tp0;
      s->ppb_req = ppb0;
      s->list_mode = lm0;
      s->persist_req = pr0;
      s->persist_set = ps0;
      s->skin = sk0;
      s->dirty = true;
      st = prepare(s);
      if (st != SRMD_OK) return st;
    }
  }
  HostState saved;
  st = save_host_state(s, &saved);
  if (st != SRMD_OK) return st;
  const int tp0 = s->tp_req, ppb0 = s->ppb_req, list0 = s->list_mode;
  const int preq0 = s->persist_req;
  const bool pset0 = s->persist_set;
  const int nmax0 = s->n_max;
  const double skin0 = s->skin;
  const int sort0 = s->sort_every;
  const bool persist0 = pset0 ? preq0 != 0 : s->persist_tuned != 0;
  int sort_trial = sort0;  // the re-sort interval of the all-pairs lists in the trials
  hipEvent_t e0, e1;
  HIPCHK(s, hipEventCreate(&e0));
  HIPCHK(s, hipEventCreate(&e1));
  int ntrials = 0;
  // one timed trial from the stored state; settings this system cannot run
  // (a skin past half a box side, the all-pairs builder over too many cells, the
  // persistent kernel where it is not available) time as 1e30
  auto trial = [&](int tp, int ppb, int list_mode, bool persistent, double skin, double *ms_per_step) -> srmd_status {
    *ms_per_step = 1e30;
    if (!skin_fits(s, skin)) return SRMD_OK;
    s->tp_req = tp;
    s->ppb_req = ppb;
    s->list_mode = list_mode;
    s->persist_set = true;
    s->persist_req = persistent ? -1 : 0;
    s->skin = skin;
    s->sort_every = sort_trial;
    s->n_max = nmax0;  // the list capacity follows the trial's skin
    s->dirty = true;
    srmd_status r = restore_host_state(s, saved);
    if (r != SRMD_OK) return r;
    r = prepare(s);
    if (r == SRMD_EINVAL) return SRMD_OK;
    if (r != SRMD_OK) return r;
    if (persistent && s->persist_groups == 0) return SRMD_OK;
    if (!s->persist_err.empty()) return SRMD_OK;
    ++ntrials;
    r = run_steps(s, 16);  // graph instantiation and the first build, untimed
    if (r != SRMD_OK) return r;
    HIPCHK(s, hipEventRecord(e0, s->stream));
    r = run_steps(s, steps_per_trial);
    if (r != SRMD_OK) return r;
    HIPCHK(s, hipEventRecord(e1, s->stream));
    HIPCHK(s, hipEventSynchronize(e1));
    Control h;
    r = read_ctl(s, &h);
    if (r != SRMD_OK) return r;
    r = check_barrier(s, &h);
    if (r != SRMD_OK) return r;
    float ms = 0.f;
    HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
    *ms_per_step = (h.error & 3) ? 1e30 : (double)ms / steps_per_trial;
    if (h.error & 3) {
      h.error &= ~3;
      r = h2d_sync(s, s->p.ctl, &h, sizeof(Control));
    }
    return r;
  };
  // the skin line search of the appendix: from start, steps of the factor 1 + step
  // up, and if the first one up is not faster, 1 - step down, until a trial is slower
  auto skin_search = [&](int tp, int ppb, int lm, bool persistent, double start, double step, double *skin_best,
                         double *t_best) -> srmd_status {
    double t0;
    srmd_status r = trial(tp, ppb, lm, persistent, start, &t0);
    double bs = start, bt = t0;
    for (int dir = 0; dir < 2 && r == SRMD_OK && bt < 1e30; ++dir) {
      const double f = dir == 0 ? 1.0 + step : 1.0 - step;
      bool better = false;
      double sk = bs * f;
      for (int k = 0; k < 16 && r == SRMD_OK; ++k, sk *= f) {
        double t;
        r = trial(tp, ppb, lm, persistent, sk, &t);
        if (r != SRMD_OK || !(t < bt)) break;
        bs = sk;
        bt = t;
        better = true;
      }
      if (better) break;
    }
    *skin_best = bs;
    *t_best = bt;
    return r;
  };
  srmd_status result = SRMD_OK;
  const double start = skin0 > 0 ? skin0 : 0.3;  // a zero skin starts from the library default
  // baseline (appendix step 2): the settings in force at the call
  double t_base = 1e30;
  result = trial(tp0, ppb0, list0, persist0, skin0 > 0 ? skin0 : start, &t_base);
  // phase I (step 3): every list method at the default layout, each with its own skin
  int dtp, dppb;
  s->tp_req = s->ppb_req = 0;
  s->persist_set = true;
  s->persist_req = 0;  // the default layout of the launch chains
  launch_of(s, &dtp, &dppb);
  // list methods: wave, thread, cell and row-staged per particle; all pairs for small systems
  auto lm_used = [&](int lm) { return lm != 4 || s->c.small_sort; };
  const int n_lm = 5;
  double t1[6] = {1e30, 1e30, 1e30, 1e30, 1e30, 1e30}, sk1[6] = {start, start, start, start, start, start};
  for (int lm = 1; lm <= n_lm && result == SRMD_OK; ++lm)
    if (lm_used(lm)) result = skin_search(dtp, dppb, lm, false, start, 0.2, &sk1[lm], &t1[lm]);
  double t1_best = 1e30;
  for (int lm = 1; lm <= n_lm; ++lm) t1_best = std::min(t1_best, t1[lm]);
  srmd_tuning best{};
  double best_t = 1e30;
  auto consider = [&](int tp, int ppb, int lm, bool persistent, double skin, double t) {
    if (t < best_t) {
      best_t = t;
      best.tp = tp;
      best.ppb = ppb;
      best.list_mode = lm;
      best.persistent = persistent ? -1 : 0;
      best.skin = skin;
    }
  };
  for (int lm = 1; lm <= n_lm; ++lm)
    if (lm_used(lm)) consider(dtp, dppb, lm, false, sk1[lm], t1[lm]);
  // phase II (step 4): methods within 20 % of the fastest; block size x t_p with the
  // stop rules of phase II of srmd_autotune, the skin re-optimised at every layout
  const int blocks[] = {64, 128, 256, 512, 1024};
  const int tp_max = s->n > 100000 ? 2 : 64;
  for (int lm = 1; lm <= n_lm && result == SRMD_OK; ++lm) {
    if (!(t1[lm] < 1e30) || t1[lm] > 1.2 * t1_best) continue;
    double skin_last = sk1[lm];
    double prev_block_best = 1e300, lm_best = t1[lm];
    for (int bi = 0; bi < 5 && result == SRMD_OK; ++bi) {
      const int bsz = blocks[bi];
      double block_best = 1e300;
      int slower = 0;
      for (int tp = 1; tp <= tp_max && tp <= bsz && result == SRMD_OK; tp <<= 1) {
        double t, sk;
        result = skin_search(tp, bsz / tp, lm, false, skin_last, 0.1, &sk, &t);
        if (result != SRMD_OK) break;
        if (t < 1e30) skin_last = sk;
        if (t < block_best) {
          block_best = t;
          slower = 0;
        } else {
          ++slower;
        }
        consider(tp, bsz / tp, lm, false, sk, t);
        lm_best = std::min(lm_best, t);
        if (slower >= 3 || t > 1.05 * block_best) break;
      }
      if (block_best > 1.10 * std::min(lm_best, prev_block_best) && bi > 0) break;
      prev_block_best = std::min(prev_block_best, block_best);
    }
  }
  // the persistent kernel (MI355X): the t_p loop at 256-thread virtual blocks for the
  // best list method so far, the skin re-optimised from the best skin
  if (result == SRMD_OK && s->prec == SRMD_PREC_F32 && best_t < 1e30) {
    const int lm = best.list_mode;
    double skin_last = best.skin, pbest = 1e300;
    int slower = 0;
    for (int tp = 1; tp <= 64 && result == SRMD_OK; tp <<= 1) {
      double t, sk;
      result = skin_search(tp, 256 / tp, lm, true, skin_last, 0.1, &sk, &t);
      if (result != SRMD_OK || !(t < 1e30)) break;
      skin_last = sk;
      if (t < pbest) {
        pbest = t;
        slower = 0;
      } else {
        ++slower;
      }
      consider(tp, 256 / tp, lm, true, sk, t);
      if (slower >= 3 || t > 1.05 * pbest) break;
    }
  }
  // step 5: with the all-pairs lists chosen, the interval of their periodic spatial
  // re-sort (in list builds; 0: never), a single minimum from the longest interval down
  best.sort_every = sort0;
  if (result == SRMD_OK && best_t < 1e30 && best.list_mode == 4) {
    const int intervals[] = {0, 64, 16, 4, 1};
    for (int q = 0; q < 5 && result == SRMD_OK; ++q) {
      if (intervals[q] == best.sort_every) continue;
      sort_trial = intervals[q];
      double t;
      result = trial(best.tp, best.ppb, 4, best.persistent != 0, best.skin, &t);
      if (result != SRMD_OK) break;
      if (t < best_t) {
        best_t = t;
        best.sort_every = intervals[q];
      } else if (intervals[q] < best.sort_every || best.sort_every == 0) {
        if (q > 1) break;  // past the minimum
      }
    }
    sort_trial = best.sort_every;
  }
  // step 7: the chosen set, timed as the baseline was
  double t_final = 1e30;
  if (result == SRMD_OK && best_t < 1e30)
    result = trial(best.tp, best.ppb, best.list_mode, best.persistent != 0, best.skin, &t_final);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tp_req = tp0;
  s->ppb_req = ppb0;
  s->list_mode = list0;
  s->persist_req = preq0;
  s->persist_set = pset0;
  s->skin = skin0;
  s->sort_every = sort0;
  s->n_max = nmax0;
  if (result == SRMD_OK && !(best_t < 1e30)) result = fail(s, SRMD_ESTATE, "no trial of the autotuner completed");
  if (result == SRMD_OK) apply_tuning(s, best);
  s->dirty = true;
  srmd_status r2 = restore_host_state(s, saved);
  if (result == SRMD_OK) result = r2;
  if (result == SRMD_OK) result = prepare(s);
  if (result != SRMD_OK) return result;
  best.baseline_ms_per_step = t_base < 1e30 ? t_base : 0.0;
  best.tuned_ms_per_step = t_final < 1e30 ? t_final : 0.0;
  best.trials = ntrials;
  best.from_cache = 0;
  if (cache_path) {
    st = srmd_tuning_cache_store(cache_path, &key, &best);
    if (st != SRMD_OK) return fail(s, st, srmd_last_error(nullptr));
  }
  if (out) *out = best;
  return SRMD_OK;
}

srmd_status srmd_batch_create(srmd_batch **out, srmd_system *const *systems, int32_t count) {
  return srmd_batch_create_limited(out, systems, count, 0);
}

srmd_status srmd_batch_create_limited(srmd_batch **out, srmd_system *const *systems, int32_t count,
                                      int32_t max_workgroups) {
  if (!out) return bfail(nullptr, SRMD_EINVAL, "out is NULL");
  if (max_workgroups < 0) return bfail(nullptr, SRMD_EINVAL, "max_workgroups must be >= 0");
  *out = nullptr;
  if (!systems || count < 1) return bfail(nullptr, SRMD_EINVAL, "need at least one system");
  for (int r = 0; r < count; ++r) {
    srmd_system *s = systems[r];
    if (!s) return bfail(nullptr, SRMD_EINVAL, "NULL system in the batch");
    for (int q = 0; q < r; ++q)
      if (systems[q] == s) return bfail(nullptr, SRMD_EINVAL, "a system appears twice in the batch");
    if (!s->integrator_set) return bfail(nullptr, SRMD_EINVAL, "every replica needs an integrator");
    if (s->prec != SRMD_PREC_F32) return bfail(nullptr, SRMD_EUNSUPPORTED, "batched replicas use float32 positions");
    srmd_status st = prepare(s);
    if (st != SRMD_OK) return bfail(nullptr, st, s->err);
    if (s->n > batch_max_particles() || !s->c.small_sort)
      return bfail(nullptr, SRMD_EUNSUPPORTED, "a batched replica must have at most 8192 particles and 8192 cells");
  }
  srmd_batch *b = new (std::nothrow) srmd_batch();
  if (!b) return bfail(nullptr, SRMD_ENOMEM, "host allocation failed");
  b->sys.assign(systems, systems + count);
  b->stream = systems[0]->stream;
  b->tp = systems[0]->tp;
  b->method = kmethod(systems[0]);
  int nmax = 0;
  for (auto *s : b->sys) nmax = std::max(nmax, s->n);
  b->lds = batch_lds_bytes(nmax);
  b->host_desc.assign((size_t)count, ReplicaDesc{});
  std::memset(b->host_desc.data(), 0xff, sizeof(ReplicaDesc) * (size_t)count);  // forces the first upload
  b->desc_buf = raw_alloc(sizeof(ReplicaDesc) * (size_t)count);
  b->d_desc = (ReplicaDesc *)b->desc_buf.ptr;
  if (!b->d_desc) {
    srmd_batch_destroy(b);
    return bfail(nullptr, SRMD_ENOMEM, "batch descriptor allocation failed");
  }
  b->max_wg = max_workgroups;
  srmd_status st = batch_replan(b);
  if (st != SRMD_OK) {
    std::string m = b->err;
    srmd_batch_destroy(b);
    return bfail(nullptr, st, m);
  }
  *out = b;
  return SRMD_OK;
}

srmd_status srmd_batch_step(srmd_batch *b, int64_t nsteps, int32_t thermo_every, srmd_thermo *trace,
                            int64_t trace_cap) {
  if (!b) return bfail(nullptr, SRMD_EINVAL, "batch is NULL");
  if (nsteps < 0 || nsteps > (1LL << 30)) return bfail(b, SRMD_EINVAL, "nsteps out of range");
  if (thermo_every < 0 || trace_cap < 0 || (trace_cap > 0 && !trace)) return bfail(b, SRMD_EINVAL, "invalid trace");
  if (nsteps == 0) return SRMD_OK;
  const long long cap = thermo_every > 0 ? trace_cap : 0;
  for (auto *s : b->sys) {
    srmd_status st = ensure_trace(s, cap);
    if (st == SRMD_OK) st = alloc_snapshot(s);
    if (st != SRMD_OK) return bfail(b, st, s->err);
  }
  srmd_status st = batch_sync_desc(b);
  if (st != SRMD_OK) return st;
  std::vector<hipStream_t> streams;
  for (auto *s : b->sys) {
    // trace settings and replay snapshot in one launch, then a host-requested
    // rebuild's spatial sort, both on the system's stream before the batched launch
    if (launch_call_begin(s->stream, s->c, s->p, s->snap, s->cur, thermo_every, cap) != hipSuccess)
      return bfail(b, SRMD_EHIP, "replica call start failed");
    st = flush_host_sort(s);
    if (st != SRMD_OK) return bfail(b, st, s->err);
    if (std::find(streams.begin(), streams.end(), s->stream) == streams.end()) streams.push_back(s->stream);
  }
  for (hipStream_t q : streams)
    if (hipStreamSynchronize(q) != hipSuccess) return bfail(b, SRMD_EHIP, "replica stream sync failed");
  hipError_t e = hipSuccess;
  for (size_t r = 0; r < b->sys.size() && e == hipSuccess; ++r)
    if (b->pieces[r] > 1) e = hipMemsetAsync(b->sys[r]->p.bar_flags, 0, sizeof(unsigned) * 2 * 256, b->stream);
  for (long long done = 0; done < nsteps && e == hipSuccess;) {
    // launches of kPersistChunk steps (an even count: every launch starts on the
    // position buffer of the call start, which the descriptors hold)
    const int cnt = (int)std::min<long long>(kPersistChunk, nsteps - done);
    e = launch_multi(b->tp, b->method, false, b->nwg, b->lds, b->stream, b->d_desc, b->d_jobs, b->d_job_off, cnt,
                     b->cooperative);
    if (e == hipSuccess && done + cnt < nsteps)
      for (size_t r = 0; r < b->sys.size() && e == hipSuccess; ++r)
        if (b->pieces[r] > 1) e = hipMemsetAsync(b->sys[r]->p.bar_flags, 0, sizeof(unsigned) * 2 * 256, b->stream);
    done += cnt;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, SRMD_EHIP, std::string("batched run: ") + hipGetErrorString(e));
  // a replica whose list overflowed is restored to the call start, its capacity
  // doubled, and replayed on its own (the single-system path follows the batched
  // trajectory bit for bit); the other replicas keep their batched result
  srmd_status result = SRMD_OK;
  for (size_t r = 0; r < b->sys.size(); ++r) {
    srmd_system *s = b->sys[r];
    st = read_ctl(s, s->h_ctl);
    if (st != SRMD_OK) return bfail(b, st, s->err);
    Control h = *s->h_ctl;
    st = check_barrier(s, &h);
    if (st != SRMD_OK) {
      if (result == SRMD_OK) result = bfail(b, st, std::string("replica ") + std::to_string(r) + ": " + s->err);
      continue;
    }
    if (h.error & 2) {
      st = restore_and_regrow(s, s->cur);
      if (st == SRMD_OK) st = run_with_replay(s, nsteps, thermo_every, cap);
    } else {
      s->cur ^= (int)(nsteps & 1);
      if (h.error & 1) st = fail(s, SRMD_ESTATE, "non-finite force or position during the run");
    }
    if (st == SRMD_OK) st = download_trace(s, cap, trace ? trace + r * (size_t)cap : nullptr);
    if (st != SRMD_OK && result == SRMD_OK) result = bfail(b, st, std::string("replica ") + std::to_string(r) + ": " + s->err);
  }
  return result;
}

srmd_status srmd_batch_autotune(srmd_batch *b, int32_t steps_per_trial, int32_t *tp_out, int32_t *ppb_out) {
  if (!b) return bfail(nullptr, SRMD_EINVAL, "batch is NULL");
  if (steps_per_trial < 1) return bfail(b, SRMD_EINVAL, "steps_per_trial must be >= 1");
  const size_t R = b->sys.size();
  // the stored configuration every trial starts from (paper appendix)
  std::vector<HostState> saved(R);
  for (size_t r = 0; r < R; ++r) {
    srmd_system *s = b->sys[r];
    srmd_status st = prepare(s);
    if (st == SRMD_OK) st = save_host_state(s, &saved[r]);
    if (st != SRMD_OK) return bfail(b, st, s->err);
  }
  // replicas in size buckets (quartiles of N): each bucket gets its own block size
  std::vector<int> order(R);
  for (size_t r = 0; r < R; ++r) order[r] = (int)r;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->sys[x]->n < b->sys[y]->n; });
  const int nb = (int)std::min<size_t>(4, R);
  std::vector<int> bucket(R);
  for (size_t q = 0; q < R; ++q) bucket[(size_t)order[q]] = (int)(q * (size_t)nb / R);
  const int kThreads[] = {64, 128, 256, 512, 1024};
  auto ok_shape = [](int tp, int threads) { return threads % tp == 0 && threads >= tp && threads <= 1024; };
  // one timed trial: every replica at threads-per-block thr[bucket] and tp, from the stored state
  auto trial = [&](int tp, const std::vector<int> &thr, double *ms) -> srmd_status {
    for (size_t r = 0; r < R; ++r) {
      srmd_system *s = b->sys[r];
      s->tp_req = tp;
      s->ppb_req = thr[(size_t)bucket[r]] / tp;
      s->dirty = true;
      srmd_status st = restore_host_state(s, saved[r]);
      if (st == SRMD_OK) st = prepare(s);
      if (st != SRMD_OK) return bfail(b, st, s->err);
    }
    b->tp = tp;
    srmd_status st = batch_replan(b);
    if (st == SRMD_EUNSUPPORTED) {  // a resource limit: this shape cannot run
      *ms = 1e30;
      return SRMD_OK;
    }
    if (st != SRMD_OK) return st;
    st = srmd_batch_step(b, std::min(steps_per_trial, 50), 0, nullptr, 0);  // first build, untimed
    if (st != SRMD_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    st = srmd_batch_step(b, steps_per_trial, 0, nullptr, 0);
    if (st != SRMD_OK) return st;
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / steps_per_trial;
    return SRMD_OK;
  };
  std::vector<int> thr((size_t)nb, 256);
  int best_tp = 0;
  double best = 1e30;
  // t_p from 1 up at 256 threads per block; the appendix's stop rules: three trials in
  // a row slower than the best, or one 5 % slower, or a resource limit
  int worse = 0;
  for (int tp = 1; tp <= 64; tp *= 2) {
    if (!multi_max_groups(tp, b->method, false, b->lds)) break;
    double ms;
    srmd_status st = trial(tp, thr, &ms);
    if (st != SRMD_OK) return st;
    if (ms >= 1e30) break;
    if (ms < best) {
      best = ms;
      best_tp = tp;
      worse = 0;
    } else if (++worse >= 3 || ms > 1.05 * best) {
      break;
    }
  }
  if (!best_tp) return bfail(b, SRMD_EUNSUPPORTED, "no thread layout of the batch could run");
  // threads per block per bucket (the appendix's p_b loop; replicas of one bucket share
  // it), the rest fixed at their best; a bucket's loop stops 10 % above its best
  for (int k = 0; k < nb; ++k) {
    int best_thr = thr[(size_t)k];
    for (int t : kThreads) {
      if (t == best_thr || !ok_shape(best_tp, t)) continue;
      std::vector<int> cand = thr;
      cand[(size_t)k] = t;
      double ms;
      srmd_status st = trial(best_tp, cand, &ms);
      if (st != SRMD_OK) return st;
      if (ms < best) {
        best = ms;
        best_thr = t;
      } else if (ms > 1.10 * best && t > best_thr) {
        break;
      }
    }
    thr[(size_t)k] = best_thr;
  }
  // the chosen layout becomes each replica's launch shape; the stored state is put back
  for (size_t r = 0; r < R; ++r) {
    srmd_system *s = b->sys[r];
    s->tp_req = best_tp;
    s->ppb_req = thr[(size_t)bucket[r]] / best_tp;
    s->dirty = true;
    srmd_status st = restore_host_state(s, saved[r]);
    if (st == SRMD_OK) st = prepare(s);
    if (st != SRMD_OK) return bfail(b, st, s->err);
    if (ppb_out) ppb_out[r] = s->ppb_req;
  }
  b->tp = best_tp;
  srmd_status st = batch_replan(b);
  if (st != SRMD_OK) return st;
  if (tp_out) *tp_out = best_tp;
  return SRMD_OK;
}

srmd_status srmd_batch_destroy(srmd_batch *b) {
  if (!b) return SRMD_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  raw_free(b->desc_buf);
  raw_free(b->jobs_buf);
  raw_free(b->joboff_buf);
  delete b;
  return SRMD_OK;
}

const char *srmd_batch_last_error(const srmd_batch *b) { return b ? b->err.c_str() : g_thread_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Stateless force evaluation that allocates nothing: every intermediate array of
// the force path (sorted copies, cell starts, neighbour list, block partials,
// control block and record) lives in one static device array per GPU.

namespace {

constexpr size_t kDirectScratchBytes = (size_t)16 << 20;  // 16 MiB per GPU
constexpr int kDirectMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kDirectScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kDirectMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device with that
// device current (the array's host-side name is not a device address).
srmd_status direct_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, SRMD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kDirectMaxDevices) return fail(nullptr, SRMD_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, SRMD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SRMD_OK;
}

// Consecutive 256-byte aligned pieces of the scratch array (host arithmetic only).
struct Carve {
  char *base;
  size_t off;
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *q = reinterpret_cast<T *>(base + off);
    off += sizeof(T) * count;
    return q;
  }
};

}  // namespace

extern "C" srmd_status srmd_compute_forces_noalloc(const srmd_lj_config *cfg, const float *d_pos,
                                                   const int32_t *d_type, float *d_force, double *d_energy,
                                                   int32_t *d_status, void *hip_stream) {
  if (!cfg || !d_pos || !d_type || !d_force || !d_energy || !d_status)
    return fail(nullptr, SRMD_EINVAL, "cfg and every device pointer are required");
  const int n = cfg->n, nt = cfg->ntypes;
  if (n < 2) return fail(nullptr, SRMD_EINVAL, "need at least 2 particles");
  if (nt < 1 || nt > kMaxTypes) return fail(nullptr, SRMD_EINVAL, "ntypes must be in 1..4");
  if (cfg->method < SRMD_CUT_TRUNC || cfg->method > SRMD_CUT_SF) return fail(nullptr, SRMD_EINVAL, "unknown cutoff method");
  if (!(cfg->skin >= 0) || !std::isfinite(cfg->skin)) return fail(nullptr, SRMD_EINVAL, "skin must be >= 0");
  // the system the force path would build for these parameters (host only)
  srmd_system t;
  t.n = n;
  t.ntypes = nt;
  for (int k = 0; k < 3; ++k) {
    if (!(cfg->box[k] > 0) || !std::isfinite(cfg->box[k]) || !std::isfinite((float)cfg->box[k]))
      return fail(nullptr, SRMD_EINVAL, "box sides must be positive and finite");
    t.Lf[k] = (float)cfg->box[k];
  }
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      const int q = a * nt + b, r = b * nt + a;
      const double sg = cfg->sigma[q], ep = cfg->epsilon[q], rc = cfg->rcut[q];
      if (!(sg > 0) || !(ep >= 0) || !(rc > 0) || !std::isfinite(sg) || !std::isfinite(ep) || !std::isfinite(rc))
        return fail(nullptr, SRMD_EINVAL, "sigma, rcut > 0 and epsilon >= 0 must be finite");
      if (sg != cfg->sigma[r] || ep != cfg->epsilon[r] || rc != cfg->rcut[r])
        return fail(nullptr, SRMD_EINVAL, "pair parameters must be symmetric");
      t.sigma[q] = sg;
      t.eps[q] = ep;
      t.rc[q] = rc;
      t.pair_given[q] = true;
    }
  t.method = cfg->method;
  t.pot = 0;
  t.skin = cfg->skin;
  if (fill_const(&t) != SRMD_OK) return fail(nullptr, SRMD_EINVAL, t.err);
  SysConst c = t.c;
  if (!c.small_sort)
    return fail(nullptr, SRMD_EUNSUPPORTED, "the allocation-free force path takes at most 8192 particles and 8192 cells");
  void *base = nullptr;
  srmd_status st = direct_scratch(&base);
  if (st != SRMD_OK) return st;
  const size_t N = (size_t)n;
  const int threads = t.tp * t.ppb;
  const int blocks = step_blocks(&t);
  SysPtrs p{};
  Carve cv{(char *)base, 0};
  p.pos[0] = cv.take<float4>(N);
  p.pos[1] = cv.take<float4>(N);
  p.vel = cv.take<float4>(N);
  p.img = cv.take<int4>(N);
  p.force = cv.take<float4>(N);
  p.wpart = cv.take<float>(N);
  p.last = cv.take<float4>(N);
  p.nnb = cv.take<int>(N);
  p.t_pos = cv.take<float4>(N);
  p.t_vel = cv.take<float4>(N);
  p.t_img = cv.take<int4>(N);
  p.cell_start = cv.take<unsigned>((size_t)c.ncell + 1);
  p.part = cv.take<BlockPartial>((size_t)blocks);
  p.ctl = cv.take<Control>(1);
  p.thermo = cv.take<Thermo>(1);
  // the list takes what is left, as many rows as fit (at most one per particle)
  const size_t used = (cv.off + 255) & ~(size_t)255;
  if (used >= kDirectScratchBytes) return fail(nullptr, SRMD_EUNSUPPORTED, "system too large for the scratch array");
  const long long rows_fit = (long long)((kDirectScratchBytes - used) / (sizeof(int) * (size_t)c.nvp)) / 64 * 64;
  const long long rows = std::min<long long>(rows_fit, (long long)c.nvp);
  if (rows < c.n_max)
    return fail(nullptr, SRMD_EUNSUPPORTED, "the neighbour list of this system does not fit the scratch array");
  c.n_max = (int)rows;
  p.nbl = cv.take<int>((size_t)rows * (size_t)c.nvp);
  if (cv.off > kDirectScratchBytes) return fail(nullptr, SRMD_EUNSUPPORTED, "system too large for the scratch array");
  hipStream_t stream = (hipStream_t)hip_stream;
  auto chk = [&](hipError_t e, const char *what) {
    return e == hipSuccess ? SRMD_OK : fail(nullptr, SRMD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  if ((st = chk(launch_direct_init(stream, c, p, d_pos, d_type, d_status), "set-up kernel")) != SRMD_OK) return st;
  if ((st = chk(launch_host_sort(stream, c, p, 0), "spatial sort")) != SRMD_OK) return st;
  if ((st = chk(launch_rebuild(stream, c, p, 0), "list build")) != SRMD_OK) return st;
  if ((st = chk(launch_force(t.tp, (int)t.method, blocks, threads, stream, c, p, 0), "force kernel")) != SRMD_OK)
    return st;
  if ((st = chk(launch_finish(1, blocks, 0, stream, c, p), "reduction")) != SRMD_OK) return st;
  return chk(launch_direct_out(stream, c, p, d_force, d_energy, d_status), "output kernel");
}
