/*
 * srmd.h -- C-ABI of libsrmd, a short-range molecular-dynamics library for one
 * AMD MI355X (gfx950) GPU.
 *
 * The library implements the data-parallel hot path of the method of
 * Bailey et al., "RUMD: A general purpose molecular dynamics package optimized to
 * utilize GPU hardware down to a few thousand particles" (arXiv:1506.05094):
 * Lennard-Jones pair forces over a Verlet neighbour list (paper section 5, force
 * kernel figure), the list built from cells after a spatial sort of all particle
 * data (section 7, cell-list figure), rebuilt on the device once any particle
 * has moved more than half the skin (section 6), and a leapfrog NVE or
 * Nose-Hoover NVT integrator (section 2, integrators).  The verbs follow the
 * paper's Python example (section 2 figure: create a simulation from a
 * configuration, set a pair potential with a cutoff method and parameters,
 * set an integrator, run n steps).
 *
 * Conventions for every call:
 *  - Host arrays are caller-owned; they are read or written during the call only.
 *  - Device memory is library-owned; it is obtained through the allocator hook
 *    (srmd_set_allocator) or hipMalloc when no hook is installed.
 *  - Every call returns an srmd_status.  Nothing aborts or throws across the ABI.
 *    After a failure, srmd_last_error(s) (or srmd_last_error(NULL) for failures
 *    without a system) returns a message.
 *  - Per-particle arrays passed in or out are in the caller's ORIGINAL particle
 *    order (index = particle id), even though the library reorders particles
 *    spatially on the device at every list rebuild.
 *  - Positions live in the periodic box [-L/2, L/2) per axis.  Box sides are
 *    stored as float32; the float32 value of each side is the box the library
 *    simulates (srmd_get_box returns it).
 *  - A system is used from one host thread at a time.  Work is enqueued on the
 *    system's HIP stream; calls that return results synchronise that stream.
 */
#ifndef SRMD_H
#define SRMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srmd_system srmd_system; /* opaque, library-owned */
typedef struct srmd_batch srmd_batch;   /* opaque, library-owned */

typedef enum {
  SRMD_OK = 0,
  SRMD_EINVAL = -1,      /* invalid argument or call order */
  SRMD_ENOMEM = -2,      /* device or host allocation failed */
  SRMD_EHIP = -3,        /* a HIP runtime call failed */
  SRMD_ESTATE = -4,      /* non-finite state detected on the device */
  SRMD_EUNSUPPORTED = -5 /* valid request this build does not support */
} srmd_status;

/* Cutoff methods of paper section 2 ("cutoff methods"): plain truncation,
 * truncation with the potential shifted to zero at r_c, truncation with the force
 * shifted to zero at r_c (a linear term added to the potential). */
typedef enum { SRMD_CUT_TRUNC = 0, SRMD_CUT_SP = 1, SRMD_CUT_SF = 2 } srmd_cutoff;

/* Position precision.  F32: float32 positions.  F32_KAHAN: float32 positions with
 * a compensated (Kahan) position update.  F64POS: float64 master positions updated
 * in float64, with a float32 copy used by the list build and the force kernel.
 * Pair forces are float32 in every variant; energy, virial, kinetic-energy and
 * displacement reductions are float64 in every variant. */
typedef enum { SRMD_PREC_F32 = 0, SRMD_PREC_F32_KAHAN = 1, SRMD_PREC_F64POS = 2 } srmd_precision;

/* Thermodynamic record of one integer time step n (all float64):
 *  pe          potential energy: half the sum of pair energies (paper, force
 *              kernel figure: compensation for double counting);
 *  ke          kinetic energy of v(n) = (v(n-1/2) + v(n+1/2)) / 2;
 *  virial      W = 1/3 sum over pairs of r_ij . F_ij;
 *  temperature 2 ke / (3N - 3)   (k_B = 1);
 *  pressure    (2 ke / 3 + W) / V;
 *  xi, xi_integral  Nose-Hoover friction and its time integral at step n;
 *  h_conserved ke + pe (+ g T0 (tau^2 xi^2 / 2 + xi_integral) under Nose-Hoover);
 *  ke_half     kinetic energy of v(n+1/2);
 *  step        step index n; n_rebuilds: list builds so far; max_nbrs: longest list. */
typedef struct {
  double pe, ke, virial, temperature, pressure, xi, xi_integral, h_conserved, ke_half;
  int64_t step, n_rebuilds;
  int32_t max_nbrs, reserved;
} srmd_thermo;

/* Create a system of n >= 2 particles of ntypes types (1..4) in an orthorhombic
 * periodic box (paper section 2 figure of the Python interface: a simulation object
 * made from a configuration of particle positions, types and box).  pos: host float32 n*3 (x,y,z per particle), wrapped into
 * [-L/2, L/2) on entry.  type: host int32 n, each in [0, ntypes).  vel: host float32
 * n*3 read as v(-dt/2), or NULL for zero.  mass: host float64 per type, or NULL for
 * unit masses.  hip_stream: a hipStream_t to enqueue on, or NULL for a stream the
 * library creates.  Fails with SRMD_EINVAL on non-finite input, a type out of
 * range or a non-positive box side.  *out receives the new system. */
srmd_status srmd_create(srmd_system **out, int32_t n, int32_t ntypes, const double box[3], const float *pos,
                        const int32_t *type, const float *vel, const double *mass, srmd_precision prec,
                        void *hip_stream);

/* Release every device and host resource of s (NULL is a no-op). */
srmd_status srmd_destroy(srmd_system *s);

/* Install a device allocator used for every later device allocation (NULL alloc
 * restores hipMalloc/hipFree).  alloc(bytes, ctx) returns device memory or NULL;
 * free(ptr, ctx) releases it.  Buffers keep the allocator they were made with. */
srmd_status srmd_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*free_fn)(void *ptr, void *ctx),
                               void *ctx);

/* 12-6 Lennard-Jones between types ti and tj (symmetric): U(r) = 4 eps [(sigma/r)^12
 * - (sigma/r)^6] for r < rcut (absolute distance), modified by the cutoff method
 * (paper section 2).  All type pairs of a system share one method; a call with a
 * different method than earlier calls fails with SRMD_EINVAL.  rcut + skin must
 * stay below half of every box side. */
srmd_status srmd_set_pair_lj(srmd_system *s, int32_t ti, int32_t tj, double sigma, double epsilon, double rcut,
                             srmd_cutoff method);

/* Two-power pair potential between types ti and tj (symmetric), in place of
 * Lennard-Jones (paper section 2 lists generalised Lennard-Jones and inverse power
 * laws among the pair potentials; both have this form):
 *   U(r) = A (sigma/r)^m - B (sigma/r)^n  for r < rcut,
 * A, B >= 0, even exponents 2 <= n < m <= 48 (B = 0: an inverse power law of
 * exponent m; A = eps n/(m-n), B = eps m/(m-n): generalised Lennard-Jones), modified
 * by the cutoff method as srmd_set_pair_lj.  All type pairs of a system use one
 * potential and one method (mixing with srmd_set_pair_lj: SRMD_EINVAL).  The
 * Coulomb term does not combine with it (SRMD_EUNSUPPORTED at the next step). */
srmd_status srmd_set_pair_mie(srmd_system *s, int32_t ti, int32_t tj, double A, double B, int32_t m, int32_t n,
                              double sigma, double rcut, srmd_cutoff method);

/* Further pair potentials among those paper section 2 lists by name; the library
 * takes their textbook forms (x = r / sigma):
 *   SRMD_POT_YUKAWA         U = eps (sigma/r) exp(-kappa (r - sigma)),  params {eps, kappa},
 *                           kappa >= 0, kappa sigma <= 60 (screened Coulomb);
 *   SRMD_POT_BUCKINGHAM     U = A exp(-r/rho) - C / r^6,  params {A, rho, C}, A, C >= 0,
 *                           rho > 0 (sigma unused but must be positive);
 *   SRMD_POT_GAUSSIAN_CORE  U = eps exp(-x^2),  params {eps};
 *   SRMD_POT_DZUGUTOV       U = eps [5.82 (x^-16 - 1.28) exp(1.1/(x - 1.87)) for x < 1.87
 *                           + 1.28 exp(0.27/(x - 1.94)) for x < 1.94],  params {eps}
 *                           (smoothly zero from 1.94 sigma on: rcut = 1.94 sigma is natural);
 *   SRMD_POT_GIRIFALCO      U = -alpha [1/(x(x-1)^3) + 1/(x(x+1)^3) - 2/x^4]
 *                           + beta [1/(x(x-1)^9) + 1/(x(x+1)^9) - 2/x^10],  params {alpha, beta},
 *                           sigma = the sphere diameter, rcut > sigma.
 * Unused params entries are ignored.  Pair forces are evaluated in float32 on the
 * device (exp from the device library); energy sums in float64. */
typedef enum {
  SRMD_POT_YUKAWA = 2,
  SRMD_POT_BUCKINGHAM = 3,
  SRMD_POT_GAUSSIAN_CORE = 4,
  SRMD_POT_DZUGUTOV = 5,
  SRMD_POT_GIRIFALCO = 6
} srmd_potential;

/* One of the further potentials between types ti and tj (symmetric) in place of
 * Lennard-Jones: params holds 4 doubles (host; see srmd_potential), modified by the
 * cutoff method as srmd_set_pair_lj (paper section 2 cutoff methods: the shifts use
 * the potential's own U(rcut) and F(rcut)).  All type pairs of a system use one
 * potential kind and one method (mixing kinds, or with srmd_set_pair_lj /
 * srmd_set_pair_mie: SRMD_EINVAL).  The Coulomb term does not combine with it
 * (SRMD_EUNSUPPORTED at the next step).  rcut + skin must stay below half of every
 * box side. */
srmd_status srmd_set_pair_potential(srmd_system *s, int32_t ti, int32_t tj, srmd_potential kind,
                                    const double *params, double sigma, double rcut, srmd_cutoff method);

/* Coulomb interactions with a shifted-force cutoff (paper section 9, the molten
 * salt benchmark): charge[t] per type (host array of ntypes doubles, reduced units
 * in which the Coulomb constant is one), one cutoff rcut > 0 for every type pair.
 * Between types a and b, inside rcut,
 *   U(r) = q_a q_b (1/r - 1/rcut + (r - rcut)/rcut^2),  F(r) = q_a q_b (1/r^2 - 1/rcut^2),
 * added to the pair's Lennard-Jones term, which must use SRMD_CUT_SF (other
 * methods with charges: SRMD_EUNSUPPORTED at the next step).  Pairs are listed
 * within max(r_c,ab, rcut) + skin.  charge = NULL removes the term.  rcut + skin
 * must stay below half of every box side (SRMD_EINVAL). */
srmd_status srmd_set_coulomb_sf(srmd_system *s, const double *charge, double rcut);

/* Neighbour-list skin s >= 0: pairs within r_c,ab + s are listed (paper section 4),
 * and the list is rebuilt once any particle has moved more than s/2 since the last
 * build (section 6).  Default 0.3. */
srmd_status srmd_set_skin(srmd_system *s, double skin);

/* Leapfrog NVE with time step dt > 0 (paper section 2, integrators: NVE Verlet /
 * leap-frog; velocities are half-step velocities v(n - 1/2)). */
srmd_status srmd_set_integrator_nve(srmd_system *s, double dt);

/* Nose-Hoover NVT leapfrog (paper section 2, integrators: NVT Nose-Hoover; the
 * example's IntegratorNVT(timeStep, targetTemperature)): time step dt > 0, target
 * temperature T0 > 0, thermostat relaxation time tau > 0 (mass Q = g T0 tau^2,
 * g = 3N - 3; the paper gives no discretisation: v(n+1/2) = [v(n-1/2)(1 - xi dt/2)
 * + F/m dt] / (1 + xi dt/2), xi(n+1) = xi(n) + dt (T(n+1/2)/T0 - 1) / tau^2). */
srmd_status srmd_set_integrator_nvt(srmd_system *s, double dt, double T0, double tau);

/* Thread layout of the force kernel (paper section 4 table of code conventions):
 * tp threads per particle (power of two, 1..64) and ppb particles per block,
 * tp*ppb <= 1024 and a multiple of 64.  (0, 0) selects the value found by
 * srmd_autotune, else the built-in default: the smallest power of two tp <= 32 with
 * n * tp >= 32768 lanes (65536 in persistent mode) and tp >= E / 64 for E the mean
 * particle count within max r_c + skin (long lists, e.g. with the Coulomb term),
 * and ppb = 256 / tp. */
srmd_status srmd_set_launch(srmd_system *s, int32_t tp, int32_t ppb);

/* Choose how a list rebuild runs (tuning; the resulting list is the same).
 * sort_mode: 0 automatic, 1 the spatial sort in one workgroup's LDS (systems of up
 * to 8192 particles and 8192 cells; larger ones fall back to 2), 2 the multi-kernel
 * counting sort.  list_mode: 0 automatic, 1 one wave per particle, 2 one thread per
 * particle (the paper's section 7 layout), 3 one wave per cell (the particles of a
 * cell share one load of their stencil's candidates), 4 all pairs (the paper's
 * O(N^2) builder for small systems, section 6: every particle against every other
 * in index order, no cells and no spatial sort; systems of at most 8192 particles
 * and 8192 cells, sort_mode 0 or 1, else SRMD_EINVAL at the next step), 5 one
 * workgroup per x-row of cells (the 25 stencil rows staged in LDS one after the
 * other, each thread testing its particle's five x cells there; the section 7 thread
 * per particle with shared, coalesced candidate loads).  The persistent kernel
 * builds one wave per particle or per cell for modes 1-3 and 5, and all pairs from
 * its LDS copy of the positions for mode 4. */
srmd_status srmd_set_rebuild_path(srmd_system *s, int32_t sort_mode, int32_t list_mode);

/* The periodic spatial re-sort of the all-pairs lists (list mode 4 of
 * srmd_set_rebuild_path; the paper's appendix, step 5, for its n2 method): the
 * particles keep their order between builds, which loses the locality of the force
 * kernel's neighbour reads as they diffuse; with builds = k > 0 they are spatially
 * sorted (as the cell methods sort at every build) before list builds 0, k, 2k, ...
 * counted from the start of the run.  0 (the default): never.  Other list modes
 * ignore it.  The result is the same pair set; the order of particles and list
 * entries (and so the float32 summation order) follows the sort. */
srmd_status srmd_set_sort_interval(srmd_system *s, int32_t builds);

/* Launch chains: how much of a step the step kernel does.  0: a separate
 * one-workgroup kernel ends each step and a list kernel (which exits unless the
 * rebuild flag is set) starts it.  1: the workgroup of the step kernel that arrives
 * last ends the step: it reduces the block partials in the fixed order of the
 * separate kernel, updates the Nose-Hoover friction, writes the record, takes the
 * rebuild decision of the paper's section 6 and, for a small system, runs the
 * spatial sort of section 7.  2: as 1, and a small system with the wave-per-particle
 * or the all-pairs list builder builds its lists at the start of the step kernel
 * when the flag is set (each wave builds the lists of its block's particles), so a
 * step is one launch.  -1 (the default): the library's choice, 2 where it applies, except 0 for a
 * small system whose step grid has more than 256 workgroups (measured slower).  The
 * trajectory, records and lists are bitwise the same in every form.  Forms that do
 * not apply (blocks that are not whole 64-thread waves, LDS arrays past 60 KiB, more
 * than 8 particles per wave to build (2 with all-pairs lists), another list builder)
 * fall back to the next lower one.  The persistent kernel and batches ignore it.  Errors: SRMD_EINVAL for
 * another value. */
srmd_status srmd_set_fused_reduction(srmd_system *s, int32_t enable);

/* Run the steps of a small system as persistent launches (one launch per 500
 * steps) instead of graph-captured launch chains (three launches per step).  Small systems are bound by latency, not by
 * arithmetic (section 3); the paper keeps their whole run on the device without
 * host round trips (section 6), and this mode also removes the launch boundaries
 * between the kernels of a step.  groups = 0: launch
 * chains (the default unless srmd_autotune chose otherwise); groups = -1: persistent,
 * the library picks the number of workgroups; groups > 0: persistent with exactly
 * that many workgroups of 512 threads, all of which must fit on the device at once
 * (SRMD_EUNSUPPORTED at the next step otherwise).  Without an explicit
 * srmd_set_launch, the default tp of the persistent mode is twice that of the launch
 * chains (64k lanes instead of 32k), so switching modes then changes the layout
 * and rebuilds the list; at an explicit launch shape a switch keeps the list and the
 * trajectory continues bit for bit.  The persistent kernel separates the time steps
 * by a device-wide barrier and repeats the reductions of the launch chain in the
 * same order, so the trajectory is the same bit for bit at the same (tp, ppb).  A
 * system of at most 8192 particles and 8192 cells keeps all its positions in every
 * workgroup's LDS; a larger one reads them from device memory and runs the launch
 * chain's four-phase sort with a barrier between phases, and then needs tp <= 8.
 * The persistent kernel needs float32 positions; srmd_step on a system it cannot
 * run returns SRMD_EUNSUPPORTED while groups != 0.  A barrier
 * that does not complete within about one second (workgroups not co-resident) ends
 * the launch and the call returns SRMD_EHIP instead of hanging. */
srmd_status srmd_set_persistent(srmd_system *s, int32_t groups);

/* Read back the thread layout in use (after defaults are resolved). */
srmd_status srmd_get_launch(const srmd_system *s, int32_t *tp, int32_t *ppb);

/* Choose tp and ppb by timing short runs from a saved copy of the current state
 * (paper appendix: each trial starts from the same stored configuration): phase I
 * the list-build method at the default layout, phase II block size x tp with the
 * appendix's stop rules for every method within 5 % of phase I's fastest (two
 * methods that close can change places at another layout), and for systems the
 * persistent kernel can run (see
 * srmd_set_persistent) a phase III over tp in persistent mode.  The fastest
 * layout, list method and mode become the system's defaults; an explicit
 * srmd_set_launch / srmd_set_rebuild_path / srmd_set_persistent still wins.  The
 * state is restored afterwards.  Any output pointer may be NULL. */
srmd_status srmd_autotune(srmd_system *s, int32_t steps_per_trial, int32_t *tp_out, int32_t *ppb_out);

/* The "same user parameters" of the paper's appendix (step 8), under which tuned
 * parameters may be reused: particles of each type, density, temperature,
 * potential parameters, integrator and time step, and the GPU type.  Pair arrays
 * are row-major ntypes x ntypes in their first ntypes^2 entries; the rest is zero. */
typedef struct {
  char gpu[64];          /* device architecture name (hipDeviceProp_t::gcnArchName) */
  int32_t compute_units; /* of that device */
  int32_t precision;     /* srmd_precision */
  int32_t cutoff_method; /* srmd_cutoff; 3 with the shifted-force Coulomb term, 4 two-power potential,
                            5 an srmd_potential (its kind in potential) */
  int32_t thermostat;    /* 0 NVE, 1 Nose-Hoover NVT */
  int32_t ntypes;
  int32_t reserved;
  int64_t count[4];      /* particles of each type */
  double density;        /* N / V */
  double temperature;    /* T0 under NVT; under NVE the kinetic temperature 2 KE / (3N - 3) of the state */
  double dt;
  double sigma[16], epsilon[16], rcut[16];
  int32_t potential;        /* 0 12-6 Lennard-Jones, 1 the two-power potential, 2..6 srmd_potential */
  int32_t reserved2;
  double pot_param[16][4];  /* per type pair, the potential's parameters besides sigma and rcut
                               (two-power: A, B, m, n; srmd_potential: its params); zero for
                               Lennard-Jones */
  double charge[4];         /* Coulomb charges per type (zero without the Coulomb term) */
  double rc_coulomb;        /* Coulomb cutoff (zero without the term) */
} srmd_tuning_key;

/* Parameters chosen by srmd_autotune_full (or read back from its cache file). */
typedef struct {
  int32_t tp, ppb;                /* thread layout, as srmd_set_launch */
  int32_t list_mode;              /* list-build method, as srmd_set_rebuild_path (1..4) */
  int32_t persistent;             /* 0 launch chains, -1 the persistent kernel */
  double skin;                    /* as srmd_set_skin */
  double baseline_ms_per_step;    /* defaults before tuning (appendix step 2); 0 from the cache */
  double tuned_ms_per_step;       /* the chosen parameters (appendix step 7); 0 from the cache */
  int32_t trials;                 /* timed trials run; 0 from the cache */
  int32_t from_cache;             /* 1: read from the cache file, nothing timed */
  int32_t sort_every;             /* re-sort interval of the all-pairs lists, as srmd_set_sort_interval */
  int32_t reserved;
} srmd_tuning;

/* Fill *key with the user parameters of s (integrator and pair potential set).
 * Reads the velocities back from the device (NVE temperature); no state changes. */
srmd_status srmd_tuning_key_of(srmd_system *s, srmd_tuning_key *key);

/* Look key up in the tuned-parameter file at path (host code only, no GPU call).
 * A record matches when the GPU name, compute units, precision, cutoff method,
 * potential, integrator, type count and particle counts are equal, dt, density,
 * every pair parameter, charge and the Coulomb cutoff agree to 1e-6 relative, and
 * the temperature to 2 % relative;
 * the last matching record wins.  *found = 1 and *out filled on a match, else
 * *found = 0.  A missing file is no match; unreadable or malformed lines are
 * skipped.  SRMD_EINVAL for NULL arguments. */
srmd_status srmd_tuning_cache_find(const char *path, const srmd_tuning_key *key, srmd_tuning *out, int32_t *found);

/* Append one record (key and the tuned parameters of t) to the file at path, one
 * text line per record (host code only).  SRMD_EINVAL if the file cannot be
 * opened for appending or an argument is NULL. */
srmd_status srmd_tuning_cache_store(const char *path, const srmd_tuning_key *key, const srmd_tuning *t);

/* The autotuner of the paper's appendix with its skin optimisation and its
 * tuned-parameter file.  With cache_path non-NULL and a matching record there
 * (srmd_tuning_cache_find), the record is applied and nothing is timed.
 * Otherwise, from a saved copy of the state (every trial starts from it):
 * a baseline trial at the defaults; phase I, each list-build method at the
 * default layout with the skin optimised separately in steps of 20 %; phase II,
 * for each method within 20 % of the fastest, block size x tp with the
 * appendix's stop rules and the skin re-optimised in steps of 10 % from the
 * last optimum at every layout; for systems the persistent kernel can run, the
 * same t_p loop in persistent mode; with the all-pairs lists chosen, the re-sort
 * interval (srmd_set_sort_interval: never, 64, 16, 4, 1 builds) with a single
 * minimum (appendix step 5); a final trial of the chosen set.  A skin step
 * multiplies the current value by 1.2 or 0.8 (1.1 or 0.9) and the search
 * goes on in the direction that was faster until a trial is slower; skins that
 * would put r_c + skin past half a box side, or that the chosen list method
 * cannot run, count as slower.  The chosen layout, list method, mode and skin
 * are applied as srmd_set_launch, srmd_set_rebuild_path, srmd_set_persistent,
 * srmd_set_skin and srmd_set_sort_interval would (they override earlier explicit
 * choices), the state
 * is restored, and with cache_path non-NULL a record is appended.  out may be NULL. */
srmd_status srmd_autotune_full(srmd_system *s, int32_t steps_per_trial, const char *cache_path, srmd_tuning *out);

/* Bin, sort and rebuild the neighbour list now, whatever the displacement (paper
 * section 7: cell index of every particle, sort and rearrangement of all particle
 * data by cell, then the list of every particle from its neighbouring cells within
 * r_c + skin; section 6 for the all-pairs method of list mode 4). */
srmd_status srmd_build_neighbor_list(srmd_system *s);

/* Forces, potential energy and virial at the current positions (no time step;
 * paper section 5, the force kernel figure: each particle's force and half its pair
 * energies summed over its list, t_p threads per particle).
 * The list is rebuilt first if the displacement criterion or a parameter change
 * asks for it.  out (nullable) receives pe and virial; its other fields describe
 * the current velocities. */
srmd_status srmd_compute_forces(srmd_system *s, srmd_thermo *out);

/* Advance nsteps time steps (paper section 2 example: Run(nsteps); each step checks
 * the displacement since the last build and rebuilds the list on the device when a
 * particle moved more than half the skin, section 6, then forces, section 5, and
 * the integrator).  If thermo_every > 0, the record of every step n with
 * n % thermo_every == 0 is written to trace (caller-owned, trace_cap entries; extra
 * records are dropped).  Synchronises once at the end.  Returns SRMD_ESTATE if a
 * non-finite force or position appeared. */
srmd_status srmd_step(srmd_system *s, int64_t nsteps, int32_t thermo_every, srmd_thermo *trace,
                      int64_t trace_cap);

/* Copy the state to host arrays in original particle order (the paper's sort
 * rearranges all particle data on the device, section 7; the original order is
 * restored here); each pointer may be NULL.
 * pos, vel, force: float32 n*3; image: int32 n*3 (box crossings); pos64: float64 n*3
 * (the float64 master positions in the F64POS variant, else the float32 positions
 * widened). force holds the forces of the last force evaluation. */
srmd_status srmd_get_state(srmd_system *s, float *pos, float *vel, int32_t *image, float *force, double *pos64);

/* Per-particle terms of the pair sums, in original particle order; either pointer
 * may be NULL.  pe: float32 n, half the pair energies of each particle (the force
 * kernel figure of paper section 5 halves them against double counting), from the
 * last force evaluation (srmd_compute_forces or a time step).  virial: float32 n,
 * 1/6 sum_j r_ij . F_ij of each particle (its share of W = 1/3 sum over pairs of
 * r_ij . F_ij, paper section 2 "energy, pressure"), from the last srmd_compute_forces
 * call only (time steps do not store it; zero before the first call).  Both sum, in
 * float64, to the pe and virial of that evaluation's record up to summation order. */
srmd_status srmd_get_particle_terms(srmd_system *s, float *pe, float *virial);

/* Overwrite positions and/or velocities (original order, float32 n*3, either NULL to
 * keep), image counters are reset when pos is given.  Forces a rebuild and clears
 * the sticky error bits of the replaced state. */
srmd_status srmd_set_state(srmd_system *s, const float *pos, const float *vel);

/* Full-state checkpoint (the paper's autotuner, appendix, starts every trial from a
 * stored configuration; this is that store, exported).  srmd_save_state writes the
 * whole dynamic state into buf (caller-owned, host memory): positions, velocities,
 * image counters and particle ids, last-build positions, last forces, the float64
 * or compensation residuals of the precision variants, the neighbour list in use
 * with its lengths, the step counter, rebuild count, Nose-Hoover friction and its
 * time integral, and the last thermodynamic record, all in the device's spatially
 * sorted order.  *needed receives the size in bytes; with buf NULL only *needed is
 * written; bytes < *needed fails with SRMD_EINVAL.  Synchronises the stream.
 * The blob is an opaque host-order byte string for this library build. */
srmd_status srmd_save_state(srmd_system *s, void *buf, size_t bytes, size_t *needed);

/* Load a blob written by srmd_save_state into s, which must have the same particle
 * count, type count, precision and float32 box (SRMD_EINVAL otherwise, and on a
 * blob whose size, types or particle ids are inconsistent; s is then unchanged).
 * When s has the same list layout as the saving system (threads per particle, list
 * capacity, cell grid, list builder and list radii), the stored list is restored
 * and steps continue the saved trajectory bit for bit, also across the launch
 * chain, the persistent kernel and batches; otherwise the list is rebuilt before
 * the next force evaluation (the same physics, other summation order).  The
 * integrator and pair potential are those set on s.  Sticky error bits clear. */
srmd_status srmd_load_state(srmd_system *s, const void *buf, size_t bytes);

/* The neighbour list (paper sections 4, 6 and 7: every j within r_c,ij + skin of i,
 * both directions, strict less-than) as (id_i, id_j) pairs in original ids,
 * lexicographically sorted (the list order itself is not specified by the paper).
 * pairs holds 2*cap int32; *count receives the total number of pairs (the call fails
 * with SRMD_EINVAL, writing nothing, when cap is too small). */
srmd_status srmd_get_neighbor_pairs(srmd_system *s, int32_t *pairs, int64_t cap, int64_t *count);

/* The most recent thermodynamic record (of the last step taken, or of the last
 * srmd_compute_forces call). */
srmd_status srmd_get_thermo(srmd_system *s, srmd_thermo *out);

/* The float32 box sides in use (written as float64). */
srmd_status srmd_get_box(const srmd_system *s, double box[3]);

/* Counters of a system: steps taken, list builds, entries of the current list,
 * the longest list of the last build, the list capacity per particle, the launch
 * shape in use (tp, ppb, blocks of the step kernel), the cell grid size, the
 * workgroups of the persistent kernel (0 when steps run as launch chains), the
 * list-build method in use (1 wave per particle, 2 thread per particle, 3 wave per
 * cell, 4 all pairs, 5 row-staged threads) and, for launch chains, the form of a
 * step (0, 1 or 2, as srmd_set_fused_reduction describes them). */
typedef struct {
  int64_t steps, n_rebuilds, list_entries;
  int32_t max_nbrs, n_max, tp, ppb, blocks, ncell, persistent_groups, list_mode;
  int32_t step_form, reserved;
} srmd_stats;

srmd_status srmd_get_stats(srmd_system *s, srmd_stats *out);

/* Time the fused step kernel: run nsteps steps one launch at a time with a HIP
 * event recorded on the system's stream immediately before and after every
 * step-kernel launch.  kernel_ms receives the sum of those event intervals,
 * device_ms the same launches timed by the device clock (first block start to last
 * block end), launches the number of step kernels timed.  In persistent mode
 * (srmd_set_persistent) the steps run as launches of the persistent kernel of 500
 * steps each (the last one shorter), each timed the same way; launches is their
 * number and device_ms is 0.  The steps are real steps of the simulation (the
 * state advances).  Any output pointer may be NULL. */
srmd_status srmd_profile_step_kernel(srmd_system *s, int64_t nsteps, double *kernel_ms, double *device_ms,
                                     int64_t *launches);

/* ---- Force evaluation without allocation ---------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the force evaluation of
 * srmd_compute_forces for a 12-6 Lennard-Jones configuration given in device
 * memory, with every intermediate array (sorted copies, cell starts, neighbour list,
 * block partials) in one static device array of 16 MiB per GPU instead of
 * library-allocated buffers.  Limits: 2..8192 particles, at most 8192 cells of side
 * >= (rcut + skin) / 2, and a neighbour list that fits the array (SRMD_EUNSUPPORTED
 * otherwise, before any work is enqueued).  Everything is enqueued on hip_stream
 * (NULL: the null stream) without a host synchronisation, hipMalloc, hipFree or
 * hipMemset, so the call can be captured into a HIP graph.  All calls on one GPU
 * share its array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller; every call clears what it
 * reads before using it. */
typedef struct {
  int32_t n, ntypes;        /* particles (2..8192) and types (1..4) */
  int32_t method;           /* srmd_cutoff, for every type pair */
  int32_t reserved;
  double box[3];            /* orthorhombic box sides */
  double skin;              /* list skin >= 0 (pairs within rcut + skin are listed) */
  double sigma[16], epsilon[16], rcut[16];  /* row-major ntypes x ntypes, symmetric */
} srmd_lj_config;

/* d_pos: device float32 n*3 (x, y, z per particle; wrapped into [-L/2, L/2) as
 * srmd_create wraps them); d_type: device int32 n.  Outputs, device memory:
 * d_force float32 n*3 in the input particle order, d_energy float64 [2] = potential
 * energy and virial W, d_status int32 [1] = 0 or error bits (1 non-finite force,
 * 2 neighbour list longer than the array holds, 4 a type out of range, taken as
 * type 0).  The results equal those of srmd_compute_forces on a system created
 * from the same positions, types and parameters at its default launch shape. */
srmd_status srmd_compute_forces_noalloc(const srmd_lj_config *cfg, const float *d_pos, const int32_t *d_type,
                                        float *d_force, double *d_energy, int32_t *d_status, void *hip_stream);

/* Message of the last failure on s (or of the calling thread when s is NULL). */
const char *srmd_last_error(const srmd_system *s);

/* ---- Batched replicas --------------------------------------------------------
 * Many independent small systems advanced together by persistent launches (the
 * ensembles of small systems mentioned in the paper's introduction; the batch
 * removes the per-step launch chain that limits one small system).  The replicas
 * are cut into pieces of about the same particle count (a replica of up to about
 * 1700 particles in a 256-replica batch stays whole; larger ones are split over
 * several workgroups that synchronise by grid barriers) and the pieces are packed
 * onto the device's workgroups largest first, so that every compute unit carries
 * about the same work; every step of a call runs inside the kernel.
 * The batch borrows the systems: it runs on their own device state, so every
 * per-system call (srmd_get_state, srmd_get_thermo, srmd_step ...) stays valid
 * between batch calls, and the systems must outlive the batch.  Requirements: at
 * least one system; every system has an integrator, float32 positions, at most
 * 8192 particles and 8192 cells, and all share the cutoff method and the threads
 * per particle.  A replica advanced in a batch follows the trajectory of the same
 * system advanced alone by srmd_step bit for bit at the same (tp, ppb), however it
 * is split or packed.  Work is enqueued on the first system's stream. */

/* Create a batch over count systems (caller-owned array, copied). */
srmd_status srmd_batch_create(srmd_batch **out, srmd_system *const *systems, int32_t count);

/* As srmd_batch_create, using at most max_workgroups workgroups (0: as many as the
 * device holds at once, at most 256).  With fewer workgroups than pieces, a
 * workgroup runs several pieces one after the other in every step (for callers
 * that share the device, and for tests of the packing). */
srmd_status srmd_batch_create_limited(srmd_batch **out, srmd_system *const *systems, int32_t count,
                                      int32_t max_workgroups);

/* Advance every replica by nsteps steps in persistent launches of 500 steps (the
 * last one shorter).  If thermo_every > 0, replica r writes the records of its steps n with
 * n % thermo_every == 0 to trace[r * trace_cap + k], k < trace_cap (caller-owned
 * array of count * trace_cap records).  Synchronises at the end.  A replica whose
 * list overflowed (paper section 4) is restored to its state at the call start, its
 * list capacity doubled, and its steps replayed on its own by the single-system
 * path; the other replicas keep their batched result.  On a non-finite replica the
 * call returns SRMD_ESTATE after finishing every other replica. */
srmd_status srmd_batch_step(srmd_batch *b, int64_t nsteps, int32_t thermo_every, srmd_thermo *trace,
                            int64_t trace_cap);

/* Choose the batch's thread layout by timing short batched runs from a stored copy
 * of every replica's state (paper appendix: each trial starts from the same stored
 * configuration): first the threads per particle shared by all replicas (1, 2, 4,
 * ... at 256 threads per block, with the appendix's stop rules: three trials in a
 * row slower than the best, one 5 % slower, or a resource limit), then per replica
 * size bucket (the replicas in quartiles of their particle count) the threads per
 * block (64 ... 1024; particles per block = threads / tp), stopping a bucket's loop
 * 10 % above its best.  The chosen shape becomes every replica's launch shape, as
 * srmd_set_launch would set it, and the states are put back (the next step rebuilds
 * the lists).  steps_per_trial >= 1 timed batch steps per trial.  *tp_out (nullable)
 * receives tp; ppb_out (nullable, count entries) each replica's particles per block.
 * A batched replica then follows its single-system trajectory at that shape bit for
 * bit, as at any shape. */
srmd_status srmd_batch_autotune(srmd_batch *b, int32_t steps_per_trial, int32_t *tp_out, int32_t *ppb_out);

/* Release the batch (not the systems). NULL is a no-op. */
srmd_status srmd_batch_destroy(srmd_batch *b);

/* Message of the last failure of a batch call (NULL: of the calling thread). */
const char *srmd_batch_last_error(const srmd_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SRMD_H */
