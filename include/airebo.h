/*
 * airebo.h -- C ABI of the MI355X (gfx950) AIREBO library.
 *
 * The library evaluates the AIREBO hydrocarbon potential: total and per-term
 * energy, per-atom forces and the virial of a periodic (or isolated) system
 * of carbon and hydrogen atoms, and integrates it in time with velocity
 * Verlet.  The method is the one whose optimisation Hoehnerbach & Bientinesi
 * describe in "Optimizing AIREBO" (Sec. 2.1): the REBO bond-order term
 * (Sec. 2.1.1, Alg. 1 and Sec. 2.1.3), the explicit torsion term (Alg. 2) and
 * the Lennard-Jones term with its C_ij connectivity and bond-order switch
 * (Sec. 2.1.2, Alg. 3); the only input of the potential is the atom
 * positions (Sec. 1) and forces are the negative gradient (Sec. 2).
 *
 * Conventions shared by every call:
 *   - Units are LAMMPS "metal": A, eV, fs, amu.  Species code 0 = C, 1 = H.
 *   - Arrays marked "device" are GPU pointers (e.g. from torch tensors on
 *     the same device as the context); "host" arrays are CPU pointers.
 *     Positions, velocities and forces are [n][3] row-major FP64.
 *   - Calls are ordered on the HIP stream passed in (NULL = default stream);
 *     device outputs are valid after that stream is synchronised.  Calls
 *     that return device-side status (airebo_compute, airebo_nve) synchronise
 *     the stream before returning so that errors can be reported.
 *   - Every call returns 0 on success or a negative AIREBO_E_* code; the
 *     message of the last error of the calling thread is airebo_last_error().
 *     Outputs are unspecified after an error.  No exception crosses the ABI.
 *   - The caller owns every array it passes; the library never frees or
 *     keeps a caller pointer beyond the call.  A context owns its parameter
 *     copy and all scratch memory.  A context is not thread safe.
 *   - Per-atom overflow is handled inside the library and counted
 *     (airebo_stats), not returned (the paper keeps a correct slow path for
 *     every case its fast kernels do not cover, Sec. 3.2 and Sec. 4.3):
 *       * list capacities (short REBO list: 8 entries per atom, growing to
 *         32; intermediate list: 48, growing to 768; LJ list; deferred-pair
 *         queue) grow on demand: an evaluation or MD chunk that overflows one
 *         is repeated with the capacity grown;
 *       * an atom whose C_ij path map (64 atoms reachable over <= 3 bonds,
 *         kept in LDS) overflows has its pairs within 3 max R2 resolved by a
 *         sequential path search in the deferred-pair kernel.
 *     AIREBO_E_CAPACITY is returned only when a growth limit is reached.
 */
#ifndef AIREBO_H
#define AIREBO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AIREBO_OK = 0,
  AIREBO_E_ARG = -1,       /* null pointer, n < 0, bad option value            */
  AIREBO_E_PARAMS = -2,    /* parameter file missing, malformed or inconsistent */
  AIREBO_E_SPECIES = -3,   /* a species code other than 0 or 1                 */
  AIREBO_E_BOX = -4,       /* a periodic side below max(6 max R2, LJ cutoff + skin) */
  AIREBO_E_NONFINITE = -5, /* a non-finite position or result                  */
  AIREBO_E_CAPACITY = -6,  /* a neighbour or work capacity limit was exceeded  */
  AIREBO_E_DEVICE = -7     /* a HIP runtime error (message carries the code)   */
};

/* Precision of the force evaluation (the integrator is FP64 in every mode).
 * The paper names double, mixed and single modes (Sec. 4.4, Sec. 5.2) without
 * defining them; here:
 *   AIREBO_FP64    every operation in FP64.
 *   AIREBO_MIXED   FP32 arithmetic of the pair, bond-order and LJ terms on
 *                  relative vectors formed in FP64; a spline argument within
 *                  1e-3 of a knot evaluated in FP64; FP64 accumulation of
 *                  forces, energies and the virial.
 *   AIREBO_SINGLE  FP32 throughout the force evaluation: relative vectors from
 *                  positions rounded to FP32, bond weights, coordination
 *                  numbers, all term arithmetic, and the force sums (FP32
 *                  atomics); per-lane energy and virial sums are FP32 and are
 *                  combined across lanes in FP64.  Forces are handed out as
 *                  FP64 copies of the FP32 sums. */
enum { AIREBO_FP64 = 0, AIREBO_MIXED = 1, AIREBO_SINGLE = 2 };
/* Term mask.  AIREBO_TERM_REBO alone is the REBO-only potential (AIREBO
 * without its intermolecular and torsion terms, Sec. 2.1). */
enum { AIREBO_TERM_REBO = 1, AIREBO_TERM_LJ = 2, AIREBO_TERM_TORSION = 4, AIREBO_TERM_ALL = 7 };
/* Van der Waals pair form inside the LJ term (Sec. 2.1.2): Lennard-Jones, or the
 * Morse potential eps [e^{-2a(r-re)} - 2 e^{-a(r-re)}] of the AIREBO-M variant,
 * under the same C_ij, S_r / S_b blend and cutoff switch.  Morse needs the
 * parameter set's morse_eps_ / morse_re_ / morse_alpha_ records (CC, CH, HH;
 * AIREBO_E_PARAMS at context creation otherwise) and AIREBO_FP64. */
enum { AIREBO_VDW_LJ = 0, AIREBO_VDW_MORSE = 1 };

typedef struct airebo_ctx* airebo_ctx_t;
typedef struct airebo_params_set* airebo_params_t;

/* Run-time options.  Zero-initialise, then set what differs from the
 * defaults; airebo_options_default() fills the defaults. */
typedef struct {
  int32_t precision;   /* AIREBO_FP64 (default), AIREBO_MIXED or AIREBO_SINGLE       */
  int32_t term_mask;   /* AIREBO_TERM_* bits; default AIREBO_TERM_ALL                  */
  double skin;         /* neighbour-list skin in A (default 1.0)                      */
  int32_t lj_cap;      /* LJ list entries per atom; 0 = automatic (grows on demand)   */
  int32_t device;      /* HIP device ordinal (default 0)                              */
  /* launch shapes (0 = default); chosen by the autotuner for a workload class */
  int32_t bond_block;  /* threads per block of the bonded kernel: 0 or 64 (64)         */
  int32_t bond_grid;   /* blocks of the bonded kernel's persistent grid (auto)        */
  int32_t defer_block; /* threads per block of the deferred-pair kernel: 0 or 64 (64) */
  int32_t short_block; /* threads per block of the short-list kernel: 256, 512, 1024 (1024) */
  int32_t vdw;         /* AIREBO_VDW_LJ (default) or AIREBO_VDW_MORSE (AIREBO-M)      */
  int32_t lj_slack;    /* LJ list entries per atom kept free beyond the largest row when an
                          MD session sizes the list; 0 = automatic (a quarter of the
                          largest row + 32)                                             */
  int32_t queue_per_atom; /* initial deferred-pair queue entries per atom; 0 = automatic (8) */
  int32_t schedule;    /* order of the force kernels on the two streams: AIREBO_SCHED_*   */
} airebo_options;

/* Force-kernel schedules (the main stream runs the short list, the near LJ
 * pairs and the deferred pairs in that order; a second stream runs the far LJ
 * pairs and the bonded terms):
 *   AIREBO_SCHED_FAR_WITH_NEAR  the second stream starts after the short list,
 *                               so the far pairs run beside the near pairs;
 *   AIREBO_SCHED_FAR_AFTER_NEAR the second stream starts after the near pairs
 *                               and runs the bonded terms, then the far pairs,
 *                               beside the deferred pairs;
 *   AIREBO_SCHED_AUTO           the second for an FP64 evaluation of one system
 *                               of more than AIREBO_SCHED_AUTO_ATOMS atoms, the
 *                               first otherwise (mixed and single precision,
 *                               batches, small systems).
 * The result does not depend on the schedule beyond the order of the force
 * atomics. */
enum { AIREBO_SCHED_AUTO = 0, AIREBO_SCHED_FAR_WITH_NEAR = 1, AIREBO_SCHED_FAR_AFTER_NEAR = 2 };
#define AIREBO_SCHED_AUTO_ATOMS 50000

void airebo_options_default(airebo_options* opt);

/* Create a context from a parameter file (format documented in the file
 * itself: scalars, angular-spline knots, bicubic and tricubic knot tables).
 * The parameters are validated (cutoffs ordered, knots increasing, symmetric
 * tables symmetric) and copied; spline coefficients are built on the host and
 * uploaded.  Errors: AIREBO_E_ARG, AIREBO_E_PARAMS, AIREBO_E_DEVICE. */
int airebo_ctx_create(const char* param_path, const airebo_options* opt, airebo_ctx_t* out);
void airebo_ctx_free(airebo_ctx_t ctx);

/* A validated parameter set held by the caller (the model of Sec. 2.1:
 * every scalar and knot table of the parameter file), for contexts created
 * without reading a file.
 *   airebo_params_load   reads and validates a parameter file
 *   airebo_params_parse  the same from the file's text in memory: text of
 *                        len bytes, host, read only during the call
 *   airebo_params_free   releases a set (NULL is accepted)
 *   airebo_ctx_create_from_params
 *                        a context from a set; the set is copied, so it
 *                        may be freed afterwards
 * Errors: AIREBO_E_ARG, AIREBO_E_PARAMS (with the failing record in the
 * message), AIREBO_E_DEVICE. */
int airebo_params_load(const char* param_path, airebo_params_t* out);
int airebo_params_parse(const char* text, size_t len, airebo_params_t* out);
void airebo_params_free(airebo_params_t params);
int airebo_ctx_create_from_params(airebo_params_t params, const airebo_options* opt, airebo_ctx_t* out);

/* Energy, forces and virial of one configuration (Sec. 2.1, Alg. 1-3).
 *   n        number of atoms (>= 0)
 *   pos      device [n][3] positions in A; any values (wrapped internally)
 *   species  device [n] int32, 0 = C, 1 = H
 *   box      host [3] orthorhombic box lengths in A (origin 0)
 *   periodic host [3] int32 flags; a periodic side must be >= max(6 max R2, LJ cutoff
 *            + skin), i.e. 12 A and 11.2 A with the shipped parameters and skin: two
 *            reaches of a three-bond C_ij path, so that one image of an atom only
 *            is reachable over such a path (Sec. 2.1.2)
 *   energy   device [4] out: total, REBO, LJ, torsion (eV)
 *   forces   device [n][3] out: eV/A, in input order
 *   virial   device [6] out: xx yy zz xy xz yz of sum_a x_a (x) F_a (eV);
 *            positive for repulsion
 *   stream   hipStream_t or NULL
 * Neighbour lists are rebuilt on every call.  Errors: AIREBO_E_ARG,
 * AIREBO_E_SPECIES, AIREBO_E_BOX, AIREBO_E_NONFINITE, AIREBO_E_CAPACITY,
 * AIREBO_E_DEVICE. */
int airebo_compute(airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species, const double* box,
                   const int32_t* periodic, double* energy, double* forces, double* virial, void* stream);

/* airebo_compute with host pointers: pos [n][3], species [n], energy [4],
 * forces [n][3] and virial [6] all in host memory.  The inputs are copied to
 * device buffers held by the context, the outputs back; the call returns
 * when they are written (synchronous, on the null stream).  Errors as for
 * airebo_compute. */
int airebo_compute_host(airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species, const double* box,
                        const int32_t* periodic, double* energy, double* forces, double* virial);

/* airebo_compute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results, with every work buffer of the evaluation
 * taken from one static device array of 28.9 MiB that the library holds on
 * each device it runs on until the process ends (set up when the first
 * context on that device is created).  The call allocates nothing; the
 * context lends its parameters, streams and events and keeps its own
 * buffers and state (an MD session of the context is ended).
 * Limits: n <= 8192 atoms, a cell grid of at most 32768 cells (cells are at
 * least half the LJ cutoff plus skin), LJ list entries of at most 1,835,008
 * near pairs (within 3 max R2 + skin: 224 per atom at 8192 atoms) and
 * 3,145,728 far pairs (384 per atom at 8192 atoms), and 196,608 deferred
 * pairs; beyond any of them the call returns AIREBO_E_CAPACITY and does no
 * work.  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (from several threads or contexts, on different streams) race and must
 * be serialised by the caller.  Synchronous like airebo_compute.  Errors
 * as for airebo_compute. */
int airebo_compute_static(airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                          const double* box, const int32_t* periodic, double* energy, double* forces,
                          double* virial, void* stream);

/* Velocity-Verlet NVE (Sec. 2): nsteps steps of length dt_fs, updating pos
 * and vel (device [n][3], A and A/fs) in place; positions are wrapped into the
 * box whenever the neighbour lists are rebuilt (when an atom has moved more
 * than half the skin since the last build).  mass: host [2] amu of C and H.
 * thermo: device [(nsteps / thermo_every) + 1][7] rows of
 * {step, PE, KE, Etot, T, rebuilds, P}, written for step 0 and every
 * thermo_every steps (thermo may be NULL when thermo_every <= 0).  PE and
 * KE in eV, T in K, `rebuilds` the neighbour-list builds since the start of
 * the call, P the pressure in bar, (2 KE + W_xx + W_yy + W_zz) / (3 V), for
 * boxes periodic in all three directions (0 otherwise).
 * One call is one MD session (airebo_md_begin, airebo_md_run,
 * airebo_md_state, airebo_md_end): one step is captured into a HIP graph and
 * replayed in chunks of 256 steps; after each chunk every error flag is
 * read.  A list or queue overflow repeats the chunk with the capacity grown;
 * a non-finite step (AIREBO_E_NONFINITE) or another error ends the call
 * with pos and vel holding the state at the start of the failing chunk.
 * Errors as for airebo_compute. */
int airebo_nve(airebo_ctx_t ctx, int64_t n, double* pos, double* vel, const int32_t* species, const double* box,
               const int32_t* periodic, const double* mass, double dt_fs, int64_t nsteps, int64_t thermo_every,
               double* thermo, void* stream);

/* Batched form: nsys independent systems stored back to back, evaluated by
 * the same kernel launches (one launch per stage over every system's atoms).
 *   sys_off  host [nsys + 1] int64, atoms of system k are [sys_off[k], sys_off[k+1]),
 *            sys_off[0] = 0
 *   boxes    host [nsys][3] box lengths; periodic host [nsys][3] flags (each
 *            periodic side >= max(6 max R2, LJ cutoff + skin))
 *   pos, species, forces as for airebo_compute over all sys_off[nsys] atoms
 *   energy   device [nsys][4] (total, REBO, LJ, torsion); virial device [nsys][6]
 * Each system's results equal those of airebo_compute on that system alone
 * (up to summation order).  Errors as for airebo_compute. */
int airebo_batch_compute(airebo_ctx_t ctx, int32_t nsys, const int64_t* sys_off, const double* boxes,
                         const int32_t* periodic, const double* pos, const int32_t* species, double* energy,
                         double* forces, double* virial, void* stream);

/* Batched velocity Verlet: as airebo_nve over every system of the batch, the
 * whole step of all systems captured into one HIP graph.  thermo: device
 * [(nsteps / thermo_every) + 1][nsys][7] rows {step, PE, KE, Etot, T, rebuilds, P}
 * per system.  Neighbour lists of all systems are rebuilt together when any
 * atom has moved more than half the skin. */
int airebo_batch_nve(airebo_ctx_t ctx, int32_t nsys, const int64_t* sys_off, const double* boxes,
                     const int32_t* periodic, double* pos, double* vel, const int32_t* species, const double* mass,
                     double dt_fs, int64_t nsteps, int64_t thermo_every, double* thermo, void* stream);

/* Molecular-dynamics session held by the context (velocity Verlet, Sec. 2).
 * The state stays on the device between calls, so a run of k steps costs k
 * replays of the captured step and nothing else.
 *   airebo_md_begin        copies pos and vel (device [n][3], read during the
 *                          call only), sizes the lists with one evaluation,
 *                          computes the initial forces and captures one step;
 *                          arguments as for airebo_nve.  Ends any earlier
 *                          session of the context.
 *   airebo_batch_md_begin  the same for a batch (arguments as for
 *                          airebo_batch_nve).
 *   airebo_md_run          advances the session by nsteps steps; thermo as
 *                          for airebo_nve (row 0: the state before the run).
 *                          Synchronises the stream.  Overflow and error
 *                          handling as for airebo_nve; after an error the
 *                          session holds the state at the start of the
 *                          failing chunk.
 *   airebo_md_state        writes the current positions (wrapped) and
 *                          velocities into pos and vel (device [n][3]; either
 *                          may be NULL); ordered on `stream`.
 *   airebo_md_end          ends the session (keeps the context's buffers).
 * Any other call on the context (airebo_compute, ...) ends its session.
 * Errors: AIREBO_E_ARG (no session, bad arguments) and those of airebo_nve. */
int airebo_md_begin(airebo_ctx_t ctx, int64_t n, const double* pos, const double* vel, const int32_t* species,
                    const double* box, const int32_t* periodic, const double* mass, double dt_fs, void* stream);
int airebo_batch_md_begin(airebo_ctx_t ctx, int32_t nsys, const int64_t* sys_off, const double* boxes,
                          const int32_t* periodic, const double* pos, const double* vel, const int32_t* species,
                          const double* mass, double dt_fs, void* stream);
int airebo_md_run(airebo_ctx_t ctx, int64_t nsteps, int64_t thermo_every, double* thermo, void* stream);
int airebo_md_state(airebo_ctx_t ctx, double* pos, double* vel, void* stream);
void airebo_md_end(airebo_ctx_t ctx);

/* Counters of the last airebo_compute / airebo_nve call (host [16] int64):
 *   0 LJ pairs inside the cutoff (each pair once)   1 pairs with C_ij = 0
 *   2 pairs that need the modified bond order b* (inside the S_r range)
 *   3 b* pairs with dS_b != 0
 *   4 bonds                                          5 neighbour-list rebuilds
 *   6 max short neighbours of one atom               7 LJ list entries (airebo_compute)
 *   8 max LJ entries of one atom                     9 spline evaluations
 *  10 of those evaluated in FP64 near a knot (AIREBO_MIXED)
 *  11 surrogate steps that fell back to AIREBO (airebo_nn_*)
 *  12 capacity growths (short, intermediate or LJ list, queue) of the last
 *     call or MD session
 *  13 pairs handed to the sequential C_ij search because an atom's path map
 *     (64 candidates) overflowed (summed over the steps of an MD session)
 *  14 pairs evaluated by the deferred-pair kernel (0 < C_ij < 1 or inside
 *     the S_r range)
 *  15 of slot 0, the far pairs (beyond 3 max R2 + skin at the list build)
 * Slots 0-4, 9-10 and 15 refer to the last force evaluation (every step in
 * NVE). */
int airebo_stats(airebo_ctx_t ctx, int64_t* out16);
/* The same counters and more (host [n] int64; slots beyond the last filled
 * are set to 0): slots 0-15 as above, then
 *  16 far LJ list entries (of slot 7)               17 max far entries of one atom
 * Returns the number of slots filled (at most 18), or an error code. */
int airebo_stats_n(airebo_ctx_t ctx, int64_t* out, int32_t n);

/* Per-kernel timing of the velocity-Verlet path: runs nsteps steps like
 * airebo_nve (same arguments, no thermo output) but launches every kernel
 * eagerly (no graph) between a pair of HIP events on `stream`.  On return
 * ms_out[k] (host, airebo_kernel_count() doubles) holds the summed device time
 * in ms of kernel k over those steps and launches_out[k] (host int64) its
 * launch count; names come from airebo_kernel_name(k).  Errors as for
 * airebo_nve.  For measurement; the results of the run are those of
 * airebo_nve. */
int airebo_profile_nve(airebo_ctx_t ctx, int64_t n, double* pos, double* vel, const int32_t* species,
                       const double* box, const int32_t* periodic, const double* mass, double dt_fs, int64_t nsteps,
                       double* ms_out, int64_t* launches_out, void* stream);
int airebo_kernel_count(void);
const char* airebo_kernel_name(int k);

/* Measured device peaks for roofline fractions (measurement support, not
 * part of the potential).
 * airebo_peak_copy: `reps` streaming copies of `bytes` (a multiple of 32)
 *   from src to dst (device pointers, caller-owned, not overlapping) after
 *   one warm-up copy; *gbs (host) = bytes read + written per second / 1e9.
 * airebo_peak_fma: a loop of eight independent fused multiply-add chains per
 *   lane over 16 wavefronts per SIMD (FP64 when fp64 != 0, else FP32), `iters`
 *   rounds after a warm-up launch; *tflops (host) = 16 iters flops per lane
 *   per second / 1e12.  Allocates and frees its own small output buffer.
 * Both run on `stream`, synchronise it, and return 0 or an error code. */
int airebo_peak_copy(const void* src, void* dst, int64_t bytes, int32_t reps, double* gbs, void* stream);
int airebo_peak_fma(int32_t fp64, int32_t iters, double* tflops, void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate.  Not part of the paper: an approximation of the
 * potential above (Sec. 2.1) by per-atom networks, with that potential as
 * its fallback and as the reference for its error.
 *
 *   E = sum_i E_NN(G_i; s_i) + E_far
 *
 * G_i holds 112 symmetry functions of atom i.  The 64 radial ones are
 * G[s*32 + m] = sum over neighbours j of species s with r < 6 A of
 * exp(-eta (r - mu_m)^2) fc(r; 6), with mu_m = 0.8 + m 5.2/31 A and
 * eta = 1 / (2 (2 5.2/31)^2).  The 48 angular ones are
 * G[64 + 16 t + c] = 2^(1-zeta) sum over pairs j<k with s_j + s_k = t,
 * both within 3.5 A, of (1 + lam cos theta_jik)^zeta
 * exp(-eta_a (r_ij^2 + r_ik^2)) fc(r_ij; 3.5) fc(r_ik; 3.5), where
 * c = 4 log2(zeta) + 2 [lam = -1] + [eta_a = 0.05], zeta in {1, 2, 4, 8},
 * lam = +-1, eta_a in {0.005, 0.05} and fc(r; R) = (1 + cos(pi r / R)) / 2.
 *
 * E_NN(G; s) = scale * (w4 . h3 + b4) + shift[s] with
 * h_k = SiLU(W_k h_{k-1} + b_k), h_0 = (G - mean) * istd and 64 units per
 * layer.  There is one network per centre species, and each ensemble member
 * holds its own pair.  Parameters of one network are 15,617 floats in the
 * order W1 [64][112], b1 [64], W2 [64][64], b2, W3 [64][64], b3, w4 [64],
 * b4 [1].  A member holds [2][15617] (species 0, then 1).  The networks run
 * on BF16 matrix cores with FP32 accumulation.
 *
 * E_far is the LJ pair term of the context's parameters (with its outer
 * cutoff switch) times a cubic switch that rises from 0 at 5 A to 1 at 6 A.
 * It has no C_ij and no bond-order switch.  It is evaluated in FP32 on
 * FP64 pair vectors, with FP64 sums.
 *
 * Every call takes the AIREBO context whose neighbour lists and integrator
 * it uses.  Both objects must live on the same device.  Box rules and
 * errors are those of the context.  AIREBO_E_CAPACITY is returned when an
 * atom has more than 192 neighbours within 6 A or more than 48 within
 * 3.5 A.  A surrogate object is not thread safe.
 * ------------------------------------------------------------------------ */
typedef struct airebo_nn* airebo_nn_t;

/* New ensemble of nmodels (1..4) members: zero weights, mean 0, istd 1,
 * scale 1, shift 0. */
int airebo_nn_create(int32_t nmodels, int32_t device, airebo_nn_t* out);
void airebo_nn_free(airebo_nn_t nn);
/* Descriptor length (112) and floats per network (15617). */
int airebo_nn_sizes(int32_t* dim, int32_t* params_per_net);
int airebo_nn_models(airebo_nn_t nn);
/* Weights, host arrays of [nmodels][2][15617] floats.  Setting them resets
 * the optimiser state; non-finite values are rejected. */
int airebo_nn_set_params(airebo_nn_t nn, const float* host);
int airebo_nn_get_params(airebo_nn_t nn, float* host);
/* Gradient left by the last airebo_nn_gradient, same layout (host). */
int airebo_nn_get_grad(airebo_nn_t nn, float* host);
/* Input normalisation mean[112] and istd[112] (> 0), output scale (> 0) and
 * per-species shift[2] in eV, all host arrays. */
int airebo_nn_set_norm(airebo_nn_t nn, const float* mean, const float* istd, double scale, const double* shift);
int airebo_nn_get_norm(airebo_nn_t nn, float* mean, float* istd, double* scale, double* shift);
/* Column sums and sums of squares of a device descriptor array G [rows][112]
 * into mom_host[2][112] (host); synchronous. */
int airebo_nn_moments(airebo_nn_t nn, const float* G, int64_t rows, double* mom_host, void* stream);

/* Descriptors G [n][112] (device FP32) of a configuration.  Positions,
 * species, box and periodic flags are as for airebo_compute.
 * Synchronous. */
int airebo_nn_descriptors(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                          const double* box, const int32_t* periodic, float* G, void* stream);
/* Jacobian-vector product out[i][f] = sum_a dG_if/dx_a . w_a, with
 * w [n][3] and out [n][112], both device FP32.  Synchronous. */
int airebo_nn_descriptor_jvp(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                             const double* box, const int32_t* periodic, const float* w, float* out, void* stream);
/* Vector-Jacobian product for nsets (1..4) sets of descriptor gradients:
 * F[k][a] = -sum_{i,f} g[k][i][f] dG_if/dx_a.  g is [nsets][n][112] and F is
 * [nsets][n][3], both device FP32.  virial[6] (device FP64) receives the
 * virial of the mean over sets, {xx,yy,zz,xy,xz,yz}, as for airebo_compute.
 * Synchronous. */
int airebo_nn_descriptor_vjp(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                             const double* box, const int32_t* periodic, const float* g, int32_t nsets, float* F,
                             double* virial, void* stream);

/* One surrogate evaluation.  Forces are the ensemble mean plus the far field.
 * spread[i] (device FP32, optional) is the RMS over members of
 * |F_member - F_mean| for atom i.  When max_i spread > threshold (eV/A, > 0),
 * the context's AIREBO evaluation replaces energy[0], the forces and the
 * virial.  energy[4] (device) is {E used, E_NN ensemble mean, E_far,
 * E_NN spread over members}; forces [n][3] and virial[6] are device FP64.
 * info[5] (host, optional) is {E_NN mean, E_far, E_NN spread, max force
 * spread, 1 if AIREBO was used else 0}.  Synchronous. */
int airebo_nn_compute(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                      const double* box, const int32_t* periodic, double threshold, double* energy, double* forces,
                      double* virial, float* spread, double* info, void* stream);
/* Loss and gradient for one labelled configuration, for every member m:
 *   L_m = w_force sum_i |F_m,i - (f_ref_i - F_far,i)|^2 + w_energy (E_m + E_far - e_ref)^2
 * Here F_m and E_m are member m's network forces and energy, and f_ref [n][3]
 * is device FP64 (e.g. AIREBO forces).  loss[nmodels] is host output.  The
 * gradient with respect to every weight stays on the device for
 * airebo_nn_adam or airebo_nn_get_grad.  Synchronous. */
int airebo_nn_gradient(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                       const double* box, const int32_t* periodic, const double* f_ref, double e_ref, double w_force,
                       double w_energy, double* loss, void* stream);
/* One Adam step (bias-corrected) on every weight with the last gradient. */
int airebo_nn_adam(airebo_nn_t nn, double lr, double beta1, double beta2, double eps, void* stream);
/* One training step: airebo_nn_gradient on one labelled configuration,
 * then airebo_nn_adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and
 * learning rate lr.  loss[nmodels] (host) is the loss before the update.
 * Synchronous. */
int airebo_nn_train_step(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const int32_t* species,
                         const double* box, const int32_t* periodic, const double* f_ref, double e_ref,
                         double w_force, double w_energy, double lr, double* loss, void* stream);
/* Velocity Verlet with surrogate forces.  Arguments are as for airebo_nve,
 * plus the fallback threshold (see airebo_nn_compute), which is checked every
 * step on the device.  *fallbacks (host, optional) returns the number of
 * steps evaluated by AIREBO.  thermo PE is the energy used for the step. */
int airebo_nn_nve(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, double* pos, double* vel, const int32_t* species,
                  const double* box, const int32_t* periodic, const double* mass, double dt_fs, int64_t nsteps,
                  int64_t thermo_every, double* thermo, double threshold, int64_t* fallbacks, void* stream);
/* An MD session (see airebo_md_begin) driven by surrogate forces with the
 * fallback threshold of airebo_nn_nve; advance it with airebo_md_run, read
 * it with airebo_md_state, end it with airebo_md_end.  The surrogate object
 * must outlive the session. */
int airebo_nn_md_begin(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, const double* pos, const double* vel,
                       const int32_t* species, const double* box, const int32_t* periodic, const double* mass,
                       double dt_fs, double threshold, void* stream);
/* Per-kernel timing of airebo_nn_nve; output as for airebo_profile_nve. */
int airebo_nn_profile_nve(airebo_nn_t nn, airebo_ctx_t ctx, int64_t n, double* pos, double* vel,
                          const int32_t* species, const double* box, const int32_t* periodic, const double* mass,
                          double dt_fs, int64_t nsteps, double threshold, double* ms_out, int64_t* launches_out,
                          void* stream);
/* Save the weights and normalisation to a binary file; load one into a new
 * object on `device`. */
int airebo_nn_save(airebo_nn_t nn, const char* path);
int airebo_nn_load(const char* path, int32_t device, airebo_nn_t* out);
/* Check of the matrix-core lane layout: D = A B for 16x16 row-major FP32
 * device matrices.  The inputs are rounded to BF16 and the products
 * accumulated in FP32.  Asynchronous on `stream`. */
int airebo_nn_mfma_check(const float* A, const float* B, float* D, void* stream);
/* The same for the 16x16x32 BF16 tile the networks use for full 32-deep
 * slices: D [16][16] = A [16][32] B [32][16], row-major FP32 device matrices
 * rounded to BF16, FP32 accumulation.  Asynchronous on `stream`. */
int airebo_nn_mfma32_check(const float* A, const float* B, float* D, void* stream);

/* Message of the calling thread's last error ("" if none). */
const char* airebo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AIREBO_H */
