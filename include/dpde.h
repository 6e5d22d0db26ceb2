/*
 * dpde.h -- C ABI of libdpde.so: one timestep of DPDE (dissipative particle
 * dynamics with energy conservation) on an AMD MI355X (gfx950), integrated by
 * velocity-Verlet on the conservative part followed by the pair-parallel
 * fluctuation/dissipation scheme SER ("Splitting with Energy Reinjection").
 *
 * Paper: Homman, Maillet, Roussel, Stoltz, "New parallelizable schemes for
 * integrating the Dissipative Particle Dynamics with Energy Conservation",
 * arXiv:1507.06643.
 *
 * Conventions shared by every entry point
 *  - Every call returns int: DPDE_OK (0) or a negative DPDE_E* code; the
 *    thread-local message of the last failure is dpde_last_error().  No C++
 *    exception crosses the boundary.
 *  - Particle arrays are FP64.  Positions and momenta are n x 3 row-major
 *    (x,y,z of particle k at [3k..3k+2]); internal energies are n values.
 *    Row k is the particle with stable identifier k: the noise G_ij^n is keyed
 *    by these identifiers and the global step n, never by storage order.
 *  - "device" pointers are HIP device allocations (e.g. torch CUDA tensors);
 *    "host" pointers are ordinary CPU memory.  The library copies its inputs;
 *    the caller keeps ownership of every buffer it passes.
 *  - Work is issued on a stream owned by the handle.  Each entry point orders
 *    itself after the work already queued on the stream given to dpde_init
 *    and returns only once its outputs are complete (dpde_step synchronises
 *    once at the end to read the device status word).
 *  - Reduced units with k_B = 1 and d = 3 (Sec. 4.1).
 */
#ifndef DPDE_H
#define DPDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define DPDE_OK 0
#define DPDE_EINVAL (-1)     /* bad parameter, non-finite input, n < 2            */
#define DPDE_EBOX (-2)       /* a dimension holds fewer than 3 cells of side rc   */
#define DPDE_ENOMEM (-3)     /* device or host allocation failed                  */
#define DPDE_EHIP (-4)       /* HIP runtime error                                 */
#define DPDE_ENEG_EINT (-5)  /* eps_i <= 0 or T_i <= 0 during a step (Sec. 4.3,   */
                             /* Sec. 4.4.2: the reinjection can drive eps < 0)   */
#define DPDE_EEOS (-6)       /* temperature inversion failed                      */
#define DPDE_EOVERFLOW (-7)  /* a particle has more neighbours than the list cap  */
#define DPDE_ENONFINITE (-8) /* a non-finite value appeared in the state          */
#define DPDE_ERANGE (-9)     /* a pair term outside the fixed-point range of the  */
                             /* SER sums (|dp_ij| or |e_ij| >= 32 in one step)    */
#define DPDE_EIO (-10)       /* a tuning-table file could not be read or written  */

/* Precision of the pair terms. */
#define DPDE_FP64 0          /* everything in FP64                                */
#define DPDE_FP32 1          /* pair forces and noise in FP32; momenta, internal  */
                             /* energies and every conserved sum in FP64          */

/* Internal equation of state eps(theta) (eq. DPDE_internalEOS). */
#define DPDE_EOS_LINEAR 0    /* eps = cv * theta (constant heat capacity, Sec. 4.1) */
#define DPDE_EOS_EINSTEIN 1  /* eps = eos_n w/(exp(w/theta)-1) + eos_c0 theta      */

/* How theta(eps) is obtained for the nonlinear EOS. */
#define DPDE_THETA_NEWTON 0  /* Newton from the high-temperature asymptote        */
#define DPDE_THETA_MLP 1     /* surrogate network inside its training range,      */
                             /* Newton outside it                                 */
#define DPDE_THETA_MLP_NEWTON 2 /* surrogate as Newton's starting point           */

/* Fluctuation/dissipation scheme. */
#define DPDE_SCHEME_SER 0    /* Sec. 3.2.1, eqs. SER_p, SER_eint_discretization   */
#define DPDE_SCHEME_SEM 1    /* Sec. 3.1.1, eq. SEM_fd (not energy conserving)    */
#define DPDE_SCHEME_HYBRID 2 /* Sec. 3.2.2: the pairs inside one of ndom[0] x      */
                             /* ndom[1] x ndom[2] equal spatial domains (the      */
                             /* paper's processors) by SSA (Sec. 3.1.2, eq.       */
                             /* SSA_ij, exponent a = +(2 gamma_ij/m) chi dt), one  */
                             /* after the other in increasing (lo id, hi id)      */
                             /* order; then the other pairs by SER on the updated  */
                             /* state.  Results depend on the decomposition, as   */
                             /* the paper notes.  Vector model, stored increments */
                             /* only.  SSA is sequential inside a domain, so its  */
                             /* cost grows with the domain size (tens of          */
                             /* particles per domain suit the GPU); the handle    */
                             /* reserves room for n * cap / 2 intra-domain pairs  */
                             /* of 40 bytes each (cap = the list capacity).       */

/* Direction of friction and noise (Sec. 2.1). */
#define DPDE_MODEL_VECTOR 0  /* along v_ij with a 3-d Gaussian G_ij (eq. DPDE,    */
                             /* the paper's variant)                              */
#define DPDE_MODEL_PROJECTED 1 /* along e_ij = (q_i - q_j)/r_ij with one scalar   */
                             /* normal xi_ij = xi_ji per pair (the original DPDE  */
                             /* model); SEM then uses the Ito term sigma^2/m      */

/* Conservative pair potential v(r), r < rc. */
#define DPDE_POT_SOFT 0      /* (a rc/2)(1 - r/rc)^2, force a (1 - r/rc) r_hat    */
#define DPDE_POT_LJ 1        /* eq. Ep: 4 eps_lj((r_lj/r)^12 - (r_lj/r)^6) shifted */
                             /* and splined so that v(rc) = v'(rc) = 0            */

/* Length of one observable record (dpde_energies, dpde_history). */
#define DPDE_REC_LEN 12

/*
 * Parameters of one system.  Sigma is derived: sigma = sqrt(2 gamma kT_ref)
 * (eq. alternative_FDR), gamma_ij = (gamma kT_ref / 2)(1/T_i + 1/T_j)
 * (eq. DPDE_fd).  Conservative pair potential by `potential`; dissipation
 * weight chi(r) = (1 - r/rc)^2 for r < rc (eq. pot_mou).  The box is [0,box[d]) along each dimension; a periodic
 * dimension wraps positions and uses the minimum image, a non-periodic one
 * has free boundaries (its cell index is clamped to the box).
 */
typedef struct dpde_params {
  int64_t n;            /* particles (>= 2)                                     */
  double box[3];        /* box lengths; floor(box/rc) >= 3 cells per dimension  */
  double mass;          /* particle mass m > 0                                  */
  double rc;            /* cut-off radius r_cut > 0                             */
  double a;             /* conservative force amplitude (>= 0)                  */
  double gamma;         /* reference friction gamma >= 0                        */
  double kT_ref;        /* reference temperature k_B T_ref > 0                  */
  double dt;            /* timestep > 0                                         */
  double cv;            /* heat capacity of the linear EOS                      */
  double eos_n, eos_omega, eos_c0; /* Einstein EOS parameters                   */
  double eps_lj, r_lj;  /* LJ well depth and length (DPDE_POT_LJ)               */
  double skin;          /* neighbour-list skin >= 0: lists hold pairs within    */
                        /* rc + skin and are rebuilt once some particle has     */
                        /* moved more than skin/2 since the last build; the     */
                        /* trajectory does not depend on it (0: every step)     */
  uint64_t seed;        /* 64-bit noise seed                                    */
  int64_t step0;        /* initial value of the step counter n                  */
  int32_t periodic[3];  /* 1 = periodic, 0 = free                               */
  int32_t eos;          /* DPDE_EOS_*                                           */
  int32_t precision;    /* DPDE_FP64 or DPDE_FP32                               */
  int32_t theta_mode;   /* DPDE_THETA_*                                         */
  int32_t scheme;       /* DPDE_SCHEME_*                                        */
  int32_t model;        /* DPDE_MODEL_*                                         */
  int32_t potential;    /* DPDE_POT_*                                           */
  uint32_t replica;     /* folded into the noise key (seed_hi ^ replica)        */
  int32_t neighbor_cap; /* list capacity per particle (0: 64, or 96 with skin)  */
  int32_t flags;        /* DPDE_FLAG_* bits                                     */
  int32_t ndom[3];      /* Hybrid: domains per dimension (>= 1)                 */
} dpde_params;

/* flags: regenerate G_ij^n in the second SER sweep, as the paper does to avoid
 * storing the increments (Sec. 3.2.1), instead of storing dp_ij per neighbour
 * in the first sweep and reading it back (the default, which trades 24 bytes
 * per neighbour of HBM traffic for the noise generation).  Results are
 * identical bit for bit either way. */
#define DPDE_FLAG_REGENERATE_NOISE 1
/* flags: after every step replace eps_i by eps_i - (E - E0)/N, E the energy of
 * the unconstrained update and E0 that of the state given to dpde_init or
 * dpde_set_state (per replica), so that the total energy stays E0
 * (Sec. 4.2).  The records then report the projected state.  A step whose
 * projection makes some eps_i <= 0 fails with DPDE_ENEG_EINT. */
#define DPDE_FLAG_PROJECT_EINT 2

typedef struct dpde_handle dpde_handle;

/*
 * Create a system from initial state (device pointers, ID order; see above)
 * and compute F(q0), U(q0), T_i(eps0) and the initial energies.  The state
 * is that of Sec. 2.1: positions q_i, momenta p_i and internal energies
 * eps_i of the mesoparticles, with total energy
 *   E = sum_{i<j} v(r_ij) + sum_i p_i^2/(2m) + sum_i eps_i
 * conserved by the dynamics (eq. DPDE), and internal temperatures T_i =
 * theta(eps_i) from the internal EOS (eq. DPDE_internalEOS).
 * hip_stream: hipStream_t the inputs were produced on (NULL = null stream).
 * Errors: DPDE_EINVAL / DPDE_EBOX on parameters, DPDE_EINVAL on non-finite
 * inputs, DPDE_ENEG_EINT on eps <= 0, DPDE_ENOMEM, DPDE_EHIP.
 */
int dpde_init(const dpde_params* params, const double* q, const double* p, const double* eps,
              void* hip_stream, dpde_handle** out);

/*
 * Advance nsteps >= 0 timesteps n -> n+1 (Sec. 3.1 and 3.2.1): velocity-Verlet
 *   p += dt/2 F(q);  q += dt p/m;  p += dt/2 F(q_new)
 * then the fluctuation/dissipation sweeps on every neighbour pair at once
 *   dp_ij = -gamma_ij chi v_ij dt + sigma sqrt(chi) G_ij^n sqrt(dt)   (eq. SER_p)
 *   d eps_i = -1/2 sum_j dp_ij . (v_ij + (dp_i - dp_j)/(2m))
 *                                     (eq. SER_eint_discretization)
 * with the increments dp_ij stored by the first sweep and read back by the
 * second (DPDE_FLAG_REGENERATE_NOISE: G_ij^n regenerated from (ids, n) in the
 * second sweep, as in Sec. 3.2.1; the same bits either way).  Between calls
 * the state is the end of a step: states and records do not depend on how
 * the steps are split over calls (inside a call the next step's kick may run
 * at the end of the previous step's sweep 2).
 * Returns the first failure of the run (DPDE_ENEG_EINT, DPDE_EOVERFLOW,
 * DPDE_ENONFINITE, DPDE_EEOS); the state is then that of the failing step,
 * partially updated, and can still be read.
 */
int dpde_step(dpde_handle* h, int64_t nsteps);

/*
 * Observables of the current state into host out[DPDE_REC_LEN]:
 *   U, K = sum p^2/(2m), sum eps, E = U + K + sum eps, P_x, P_y, P_z,
 *   T_kin = sum p^2/m / (3(N-1)), T_int = N / sum 1/T_i, n (step counter),
 *   |grad U|^2 = sum |F_i|^2, Laplacian of U = 2 sum_{i<j} (v'' + 2 v'/r)
 * (energy of Sec. 2.1 with the kinetic term p^2/(2m); eqs. Tkin, Tint; the
 * last two give the configurational temperature of eq. Tcon as the ratio of
 * their time averages).  Each sum is exact in 128-bit fixed point before its
 * final rounding, so records do not depend on the order of the particles.
 */
int dpde_energies(dpde_handle* h, double out[DPDE_REC_LEN]);

/*
 * Per-step observable records written by the stepping calls, oldest first,
 * into host out[cap][nrep][DPDE_REC_LEN] (nrep = 1 for dpde_init handles; each
 * record as dpde_energies).  *count receives the number of steps returned:
 * the history holds the last min(65536, 2^26/(96 nrep)) steps at most.  The history is
 * cleared by the call.
 */
int dpde_history(dpde_handle* h, double* out, int64_t cap, int64_t* count);

/* Current state (q_i, p_i, eps_i of Sec. 2.1) into device buffers in ID
 * order (q, p: n x 3; eps: n); any pointer may be NULL.  *step (host)
 * receives the step counter if non-NULL. */
int dpde_get_state(dpde_handle* h, double* q, double* p, double* eps, int64_t* step);

/* Replace the state (device pointers, ID order) and the step counter; forces,
 * temperatures and energies are recomputed as in dpde_init. */
int dpde_set_state(dpde_handle* h, const double* q, const double* p, const double* eps,
                   int64_t step);

/* Conservative forces F(q) (device, n x 3, ID order) and U (host) of the
 * current positions. */
int dpde_forces(dpde_handle* h, double* F, double* U);

/* Release every resource of the handle (NULL is accepted). */
int dpde_free(dpde_handle* h);

/* Number of neighbour-list builds so far (host *builds). */
int dpde_list_builds(dpde_handle* h, int64_t* builds);

/* Thread-local description of the last failure ("" if none). */
const char* dpde_last_error(void);

/* hipStream_t the handle issues its work on (for event timing). */
void* dpde_stream(dpde_handle* h);

/*
 * Batched replicas: nrep independent systems advanced together by the same
 * launches.  params[r] gives replica r's n, box, periodic, seed and replica
 * tag; the physical parameters (mass, rc, a, gamma, kT_ref, dt, EOS,
 * precision, scheme) are taken from params[0] and must agree across replicas.
 * q, p, eps hold the replicas back to back (device, ID order inside each
 * replica): replica r occupies rows offsets[r] .. offsets[r+1]-1 with
 * offsets[0] = 0 (host array of nrep+1).  Particle identifiers, and so the
 * noise keys, are local to each replica: replica r matches a single system
 * built from params[r] bit for bit.
 */
int dpde_init_batch(const dpde_params* params, int32_t nrep, const int64_t* offsets,
                    const double* q, const double* p, const double* eps, void* hip_stream,
                    dpde_handle** out);

/* Observables of every replica into host out[nrep][DPDE_REC_LEN] (as dpde_energies). */
int dpde_energies_batch(dpde_handle* h, double* out);

/*
 * Capture nsteps steps (even, > 0) into one HIP graph and replay it reps
 * times: equivalent to dpde_step(h, nsteps * reps), with one launch per
 * replay.  The graph is cached per nsteps and captured again when nsteps,
 * the launch shape or the surrogate's weights (dpde_mlp_set, dpde_mlp_train)
 * change.
 */
int dpde_step_graph(dpde_handle* h, int64_t nsteps, int64_t reps);

/* Kernel launch shape: block size of the pair passes (64, 128, 256, 512 or 1024). */
int dpde_set_tuning(dpde_handle* h, int32_t pair_block, int32_t aux_block);

/*
 * Launch shapes of the step kernels and the form of the SER sweeps.  No
 * choice changes the trajectory beyond rounding: every launch shape gives
 * the same bits, and the two pair forms agree to rounding (their
 * per-particle sums are added in different arithmetic), so the shape can be
 * tuned on the live system.
 *   pair_block  threads per block of the lane-group pair passes (64..256)
 *   aux_block   threads per block of the per-particle passes (64..1024)
 *   pairs       form of the SER sweeps (eqs. SER_p, SER_eint_discretization):
 *     DPDE_PAIRS_BOTH_SIDES     every pair term evaluated on both of its
 *                               particles' lanes and added in FP64 in
 *                               neighbour-identifier order;
 *     DPDE_PAIRS_ONCE_PER_TILE  a pair joining two particles of one tile of
 *                               128 consecutive particles (cell order)
 *                               evaluated once for both, a pair joining two
 *                               tiles once per particle; the per-particle
 *                               sums exact in 64-bit fixed point (grid 2^-46,
 *                               a term of magnitude >= 32 fails the step with
 *                               DPDE_ERANGE), rounded once.  The default.  It
 *                               applies to SER with the soft potential whose
 *                               force and potential terms fit pass A's grid
 *                               (a < 1024 and a rc / 4 < 2^20); SEM, Hybrid,
 *                               the LJ potential and larger a run the first
 *                               form whatever this field says.
 *   order_block  memory order of the particles: sorted by cell, the cells
 *               taken in blocks of order_block^3 (compact blocks keep more of
 *               a particle's neighbours inside its tile and its cache lines).
 * Either form gives trajectories that do not depend on the memory order, the
 * skin, the rebuild schedule or the batching.  dpde_set_tuning sets the first
 * two fields only.  A change of form or order rebuilds the lists and the
 * forces from the current state.
 */
#define DPDE_PAIRS_BOTH_SIDES 0
#define DPDE_PAIRS_ONCE_PER_TILE 1
typedef struct dpde_shape {
  int32_t pair_block;
  int32_t aux_block;
  int32_t pairs;
  int32_t order_block; /* 1..8: memory order of the cells, blocks of
                          order_block^3 cells in row-major block order
                          (1: row-major cells, the default) */
} dpde_shape;
int dpde_get_shape(dpde_handle* h, dpde_shape* out);
int dpde_set_shape(dpde_handle* h, const dpde_shape* shape);

/* Autotuner: time every launch shape over `steps` steps of this system and
 * keep the fastest.  The candidates are the pair form (both forms where the
 * tile form applies), the cell order (order_block 1..4), the lane-group
 * block (64/128/256 threads: the list build and the both-sides passes) and
 * the per-particle block (128/256/512).  The winner is applied as by
 * dpde_set_shape, its pair and per-particle blocks and time per step are
 * returned (read the full shape with dpde_get_shape), and it is recorded in
 * the process's tuning table (below) for this system's size class.  The
 * state, step, list-build count and history are restored after every trial,
 * so the run continues from where it was, as it would under the chosen shape
 * (block sizes and cell order change no bit; the two pair forms agree to
 * rounding).  Allocates a snapshot (state and history) for the duration of
 * the call.  Not for use during graph capture. */
int dpde_autotune(dpde_handle* h, int32_t steps, int32_t* pair_block, int32_t* aux_block,
                  double* ms_per_step);

/*
 * Tuning table: launch shapes by size class, kept by the library for the
 * life of the process.  The key is (floor(log2 N), replica class, precision)
 * with N the particles of the handle and replica class 0 for one system,
 * 1 + floor(log2 nrep) for nrep >= 2 replicas.  dpde_autotune records its
 * winner; dpde_init and dpde_init_batch start a handle with the recorded
 * shape of its class, if any (the pair form applies where the tile form is
 * available).  The table persists through a text file, one entry per line:
 *   nclass rclass precision pair_block aux_block pairs order_block ms_per_step
 * ('#' starts a comment line).  dpde_tuning_load merges a file into the
 * table (an entry replaces one of the same key) and fails with DPDE_EIO if
 * the file cannot be opened or a line does not parse, DPDE_EINVAL if a shape
 * is out of range (the table is then unchanged).  dpde_tuning_save writes
 * the table (DPDE_EIO on failure).  dpde_tuning_lookup gives the entry for
 * (n, nrep, precision): *found = 1 and the shape and time, or *found = 0.
 * Host-only calls: they need no device.
 */
int dpde_tuning_load(const char* path);
int dpde_tuning_save(const char* path);
int dpde_tuning_clear(void);
int dpde_tuning_lookup(int64_t n, int32_t nrep, int32_t precision, dpde_shape* shape,
                       double* ms_per_step, int32_t* found);

/*
 * Per-kernel timing: when enabled, every kernel launch of dpde_step is
 * bracketed by HIP events on the handle's stream.  dpde_profile_read fills
 * names (host, nmax x 32 chars), total milliseconds and launch counts for up
 * to nmax kernels and returns how many kernels it reported; reading resets
 * the accumulators.
 */
int dpde_profile_enable(dpde_handle* h, int32_t enable);
int dpde_profile_read(dpde_handle* h, char* names, double* total_ms, int64_t* launches,
                      int32_t nmax);

/*
 * Internal temperature theta(eps) for n values (device arrays) under the
 * handle's EOS with the given DPDE_THETA_* mode (eq. DPDE_internalEOS).
 * iters (device, may be NULL) receives the Newton iterations per value.
 */
int dpde_theta(dpde_handle* h, const double* eps, double* theta, int32_t* iters, int64_t n,
               int32_t mode);

/* eps(theta) of the handle's EOS for n values (device arrays). */
int dpde_eos_energy(dpde_handle* h, const double* theta, double* eps, int64_t n);

/*
 * Surrogate network for theta(eps) of the nonlinear EOS: a 1 -> 32 -> 32 -> 1
 * perceptron with tanh hidden units on x = (ln eps - in_c)/in_s, output
 * y with theta = exp(out_c + out_s y).  Weights are packed (FP32) as
 * W1[32], b1[32], W2[32][32] (row = output unit), b2[32], W3[32], b3:
 * DPDE_MLP_NPARAM values.  Inference runs with BF16 weights and FP32
 * accumulation on the matrix cores.
 */
#define DPDE_MLP_NPARAM 1153

typedef struct dpde_mlp_cfg {
  double theta_lo, theta_hi; /* training range of theta                          */
  int64_t nsamples;          /* training samples (theta log-uniform in range)    */
  int64_t iters;             /* Adam iterations                                  */
  int32_t batch;             /* samples per iteration                            */
  int32_t pad;
  double lr;                 /* Adam step size                                   */
  uint64_t seed;             /* initialisation and sampling seed                 */
} dpde_mlp_cfg;

/* Train the surrogate on the GPU (forward, backward and Adam kernels) on
 * samples theta_k -> eps(theta_k) of the handle's EOS; loss_curve (host,
 * may be NULL) receives the loss of every iteration. */
int dpde_mlp_train(dpde_handle* h, const dpde_mlp_cfg* cfg, float* loss_curve);

/* Weights (host FP32, DPDE_MLP_NPARAM) and the 4 normalisation constants
 * {in_c, in_s, out_c, out_s} (host FP64). */
int dpde_mlp_get(dpde_handle* h, float* weights, double* norm4);
int dpde_mlp_set(dpde_handle* h, const float* weights, const double* norm4);

/* Loss and gradient (host FP32, DPDE_MLP_NPARAM) of one batch of normalised
 * inputs x and targets t (device FP32 arrays of n) under the FP32 weights. */
int dpde_mlp_grad(dpde_handle* h, const float* x, const float* t, int64_t n, float* loss,
                  float* grad);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight loops, harnesses that forbid hipMalloc): the same loss and
 * gradient as dpde_mlp_grad, bit for bit, with the block partials, the summed
 * gradient and the loss held in a fixed static device buffer of about 300 KB
 * per GPU (64 block partials of DPDE_MLP_NPARAM floats), which each GPU the
 * library runs on keeps until the process ends, instead of buffers the handle
 * allocates on first use.  The call allocates nothing; the weights must exist
 * (dpde_mlp_train or dpde_mlp_set).  1 <= n <= DPDE_MLP_GRAD_NOALLOC_MAX_N,
 * else DPDE_EINVAL.  Every call on one GPU shares that buffer: calls that
 * overlap on one GPU (several threads or streams) race and must be ordered by
 * the caller.  x, t: device FP32 arrays of n; loss, grad: host, as in
 * dpde_mlp_grad.
 */
#define DPDE_MLP_GRAD_NOALLOC_MAX_N ((int64_t)1 << 26)
int dpde_mlp_grad_noalloc(dpde_handle* h, const float* x, const float* t, int64_t n, float* loss,
                          float* grad);

/* Network output y for normalised inputs x (device FP32 arrays of n) with the
 * BF16 inference kernel. */
int dpde_mlp_eval(dpde_handle* h, const float* x, float* y, int64_t n);

/* ---- test hooks ---------------------------------------------------------- */

/* Linear cell index (within its replica) of every particle, by ID (device int32 n). */
int dpde_debug_cells(dpde_handle* h, int32_t* cell_of_id);

/* The memory order the last list build chose: for every memory slot, the
 * identifier row (the replica's first row + the particle's ID) of the particle
 * it holds (device int32 n).  The particles of one cell (side at least rc, as
 * the cells of Sec. 3.1.2) fill consecutive slots in increasing ID order. */
int dpde_debug_order(dpde_handle* h, int32_t* row_of_slot);

/* 1/T_i of every particle as the last step left it (device FP64 n, ID order):
 * the inverse temperature of eq. DPDE_internalEOS that the next step's
 * friction gamma_ij uses (eq. DPDE_fd). */
int dpde_debug_inv_temperature(dpde_handle* h, double* inv_t);

/* Length of every particle's pair list of the current step (device int32 n,
 * ID order): its neighbours within rc, less the pairs inside its tile that
 * the partner's list carries when the sweeps evaluate such pairs once
 * (DPDE_PAIRS_ONCE_PER_TILE). */
int dpde_debug_list_lengths(dpde_handle* h, int32_t* lengths);

/* Neighbour pairs (lo id, hi id) with r^2 < rc^2 of the current positions
 * (device int32 cap x 2, unordered); *npairs (host) receives the count,
 * which may exceed cap (then only cap pairs are written). */
int dpde_debug_pairs(dpde_handle* h, int32_t* lohi, int64_t cap, int64_t* npairs);

/* The four Philox-4x32-10 words and three normals G of pairs (lo[k], hi[k])
 * at step n (device arrays: raw n x 4, g n x 3 FP64, g32 n x 3 FP32; any
 * output may be NULL).  Needs no handle. */
int dpde_debug_rng(uint64_t seed, uint32_t replica, int64_t step, const uint32_t* lo,
                   const uint32_t* hi, int64_t n, uint32_t* raw, double* g, float* g32);

#ifdef __cplusplus
}
#endif
#endif /* DPDE_H */
