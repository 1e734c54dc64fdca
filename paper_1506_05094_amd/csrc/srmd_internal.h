// Internal layout shared by the kernels and the host runtime of libsrmd.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace srmd {

constexpr int kMaxTypes = 4;
constexpr int kMaxPairs = kMaxTypes * kMaxTypes;

// The cell histogram of a large system is scanned in tiles of 2^shift cells, one
// workgroup per tile, with at most kScanMaxTiles tiles (shift >= 10).
constexpr int kScanMaxTiles = 2048;
__host__ __device__ inline int scan_tile_shift(int ncell) {
  int s = 10;
  while (((ncell - 1) >> s) >= kScanMaxTiles) ++s;
  return s;
}
__host__ __device__ inline int scan_tiles(int ncell) { return ((ncell - 1) >> scan_tile_shift(ncell)) + 1; }

// Per-type-pair float32 constants of the pair kernel and of the list build.
struct PairTable {
  float cs2[kMaxPairs];    // (rc_ab + skin)^2 rounded once to float32: list radius
  float rc2[kMaxPairs];    // rc_ab^2 rounded once to float32: force cutoff
  float sig2[kMaxPairs];   // sigma^2
  float eps4[kMaxPairs];   // 4 eps
  float eps24[kMaxPairs];  // 24 eps
  float ushift[kMaxPairs]; // U(rc) for the shifted methods (0 for plain truncation)
  float fc[kMaxPairs];     // F(rc) = -U'(rc) for shifted force (0 otherwise)
  float rc[kMaxPairs];     // rc_ab
  // shifted-force Coulomb term (kernel method 3 only): q_a q_b per pair, and of the
  // one Coulomb cutoff r_cc: r_cc^2, 1 / r_cc^2 and 2 / r_cc
  float qq[kMaxPairs];
  float rcc2, inv_rcc2, two_inv_rcc;
  // two-power potential A (sigma/r)^m - B (sigma/r)^n (kernel method 4; A and m A
  // travel in eps4 and eps24): B, n B and the half exponents m/2, n/2
  float mie_b[kMaxPairs], mie_nb[kMaxPairs];
  int mie_hm[kMaxPairs], mie_hn[kMaxPairs];
  // further potentials (kernel method 5, kind in SysConst::pot_kind): four float32
  // constants per pair derived from the parameters (see pair_further)
  float gen[kMaxPairs][4];
};

// Everything a kernel needs besides pointers; passed by value.
struct SysConst {
  int n;         // particles
  int ntypes;
  int nvp;       // row stride of the list (n rounded up to 64)
  int n_max;     // list capacity per particle
  int tp;        // threads per particle the list layout is built for
  int ncell;     // nc.x * nc.y * nc.z
  int nc[3];     // cells per axis
  int full_axis; // bit k set: axis k has fewer than 5 cells, visit every cell along it
  float L[3];    // float32 box sides
  float invL[3]; // (float)(1.0 / (double)L)
  float halfL[3];
  float cscale[3]; // nc / L (float32), cell coordinate scale
  double Ld[3];    // (double)L
  float dt;        // time step (float32)
  float pad0;
  double dtd;       // time step (float64)
  double T0;        // target temperature
  double inv_tau2;  // 1 / tau^2 (0: no thermostat coupling)
  double half_skin2; // (skin / 2)^2 in float64
  double g;          // degrees of freedom 3N - 3
  double volume;
  int thermostat;    // 1: Nose-Hoover
  int small_sort;    // 1: the spatial sort runs in one workgroup (small systems)
  int list_kind;     // list builder of the launch chain: 1 wave per particle, 2 thread per particle, 3 wave per cell
  int list_blocks;   // grid of the thread-per-particle list build and the sort kernels
  int pot_kind;      // kernel method 5: 2 Yukawa, 3 Buckingham, 4 Gaussian core, 5 Dzugutov, 6 Girifalco
  int sort_every;    // all-pairs lists (list_kind 4): spatial sort at every k-th build (0: never)
  int pad1;
  float inv_mass[kMaxTypes];
  double mass[kMaxTypes];
  PairTable pt;
};

// Device-resident control words (one 256-byte block).
struct Control {
  int rebuild;       // 1: rebuild the list before the next force evaluation
  int error;         // sticky: bit 0 non-finite force/position, bit 1 list overflow,
                     // bit 2 a grid barrier of the persistent kernel timed out
  int max_nbrs;      // longest list of the last build
  int thermo_every;  // record every k-th step into the trace (0: never)
  long long step;    // steps taken
  long long n_rebuilds;
  long long n_records;     // records written to the trace
  long long trace_cap;     // capacity of the device trace
  long long list_entries;  // total entries of the current list
  double xi;               // Nose-Hoover friction at the current step
  double xi_int;           // its time integral
  unsigned long long prof_ticks;  // accumulated step-kernel durations (device clock ticks)
  long long prof_count;           // step kernels accumulated
  int resorted;                   // all-pairs lists: the build ahead starts from a fresh spatial sort
  int pad[41];
};

static_assert(sizeof(Control) == 256, "control block layout");

// Thermo accumulators of the last force evaluation / step.
struct Thermo {
  double pe, ke, virial, temperature, pressure, xi, xi_integral, h_conserved, ke_half;
  long long step, n_rebuilds;
  int max_nbrs, reserved;
};

// Per-block float64 partial sums of the step and force kernels, and the device
// clock at the block's start and end (for the kernel's duration).
struct BlockPartial {
  double pe, w, ke_half, ke_int, disp2;
  int nonfinite;
  int pad;
  unsigned long long t0, t1;
};

struct SysPtrs {
  float4 *pos[2];   // float32 positions, type bits in .w (double buffer)
  float4 *vel;      // velocities, .w unused
  int4 *img;        // image counters in .xyz, original particle id in .w
  float4 *force;    // last forces, per-particle potential energy in .w
  float *wpart;     // per-particle virial 1/6 sum_j r_ij . F_ij of the last force-only evaluation
  float4 *last;     // positions at the last build
  double *pos64;    // float64 master positions (3 per particle) or nullptr
  float4 *kahan;    // Kahan residuals or nullptr
  int *nbl;         // neighbour list, tp-interleaved column-major
  int *nnb;         // list lengths
  unsigned *cell_of;
  unsigned *slot_in_cell;
  unsigned *cell_count;
  unsigned *cell_start; // ncell + 1 entries
  unsigned *tile_count; // particles per tile of cells (kScanMaxTiles entries), for the scan
  unsigned *perm_tmp;
  float4 *t_pos;    // gather targets of the spatial sort
  float4 *t_vel;
  int4 *t_img;
  double *t_pos64;
  float4 *t_kahan;
  BlockPartial *part;
  Control *ctl;
  Thermo *thermo;   // last record
  Thermo *trace;    // device trace (trace_cap records)
  unsigned *bar_flags;  // arrival words of the persistent kernel's grid barrier (2 x 256)
  unsigned *arrive;     // arrival counters of a step kernel that ends the step itself (0 between launches)
};

// The call-start copy of a system's dynamic state, put back when a list overflow
// forces a replay of the call (pos64 and kahan only in their precision variants).
struct Snapshot {
  float4 *pos, *vel, *last, *kahan;
  int4 *img;
  double *pos64;
  Control *ctl;
};

// One system of a persistent launch: its constants, its device arrays, the position
// buffer in use at the launch and the shape of its single-system step launch.
struct ReplicaDesc {
  SysConst c;
  SysPtrs p;
  int cur;
  int G;        // blocks of the single-system step kernel (block partials per step)
  int vb;       // threads per block of that launch (a multiple of 64)
  int pad;
};

// One workgroup's share of a persistent launch: piece w of g of system rep.  A
// workgroup runs its jobs one after the other in every step; a system split over
// g > 1 workgroups synchronises them with a grid barrier, and such a job is the
// only job of its workgroups.
struct CoopJob {
  int rep, w, g, pad;
};

}  // namespace srmd
