/*
 * aap.h -- C ABI of libaap.so: one time step of the metric Vicsek-class models
 * of aligning self-propelled particles on one AMD Instinct MI355X (gfx950).
 *
 * Model (Kuersten, "Aligning Active Particles Py Package", CPC):
 *   - N point particles, state x in [0,Lx], y in [0,Ly], theta in [-pi,pi]
 *     (Sec. 2);
 *   - metric neighbourhood Omega_i = {j != i : |r_i - r_j| <= R} (Eq. (6)),
 *     with periodic images or reflecting mirror images per axis (Sec. 2.4);
 *   - Vicsek rule (VM): collision theta_i <- arg[e^{i theta_i} +
 *     sum_{Omega_i} e^{i theta_j}] + omega + eta xi, xi ~ U[-pi,pi]
 *     (Eqs. (1),(2)), then streaming r_i <- r_i + v e^{i theta_i(t+1)}
 *     (Eq. (4));
 *   - nematic Vicsek rule (NVM): as VM, but a neighbour whose orientation
 *     differs from theta_i by more than pi/2 (cos(theta_i - theta_j) < 0)
 *     enters the sum turned by pi (Eq. (3));
 *   - overdamped Langevin rule: Euler-Maruyama step of Eq. (5),
 *     theta_i <- theta_i + dt (Gamma h(|Omega_i|) sum sin(o(theta_j -
 *     theta_i)) + omega) + eta sqrt(dt) g, r_i <- r_i + v dt e^{i theta_i};
 *   - neighbour search through cell lists with a 3x3 cell scan (Sec. 3.2);
 *   - on-the-fly measurement of the polar order p, the nematic order q and
 *     the mean neighbour number nbar, moments 1..4 over the measured states,
 *     and histograms of the angles and of the neighbour numbers (Sec. 3.4);
 *   - a checkpoint of the whole simulation (state, step, measurements) that
 *     resumes with results identical to an uninterrupted run (Sec. 3.6).
 *
 * Conventions of every entry point:
 *   - status: AAP_OK (0) or a negative AAP_E* code; the library never aborts
 *     or throws across this boundary; aap_last_error() gives a message for
 *     the last failing call on the calling thread;
 *   - a handle must not be used from two threads at once;
 *   - pointers documented "host" are ordinary CPU memory owned by the
 *     caller; "device" pointers are GPU memory on the current HIP device;
 *   - work is enqueued on the HIP stream given to aap_create; calls marked
 *     "synchronous" wait for that stream before returning.
 *
 * Positions are stored in binary32; the box sides are rounded to binary32
 * once at creation and used in that form everywhere.  The decisions that
 * yield integers -- each particle's cell and each neighbour test d^2 <= R^2 --
 * are taken in binary64 from the binary32 coordinates, with a fixed sequence
 * of rounded operations, so the cell ids, the particle order and the
 * neighbour counts are reproducible exactly by an independent program.
 */
#ifndef AAP_H
#define AAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AAP_OK 0
#define AAP_EINVAL (-1)    /* bad parameter, bad pointer or call order       */
#define AAP_ENOMEM (-2)    /* workspace smaller than aap_workspace_bytes()   */
#define AAP_EHIP (-3)      /* HIP runtime error (message names it)           */

#define AAP_RULE_VM 0       /* Vicsek collision rule, Eq. (2)              */
#define AAP_RULE_LANGEVIN 1 /* overdamped Langevin alignment, Eq. (5)      */
#define AAP_RULE_NVM 2      /* nematic Vicsek collision rule, Eq. (3)      */

/*
 * Model parameters; names follow the keyword arguments of the paper's
 * aappp_init (Sec. 4).
 *   N          particle count, 1 <= N <= 2^32 - 1
 *   Lx, Ly     box sides (> 0); rounded to binary32 at creation
 *   R          interaction radius (> 0); the box must hold at least three
 *              cells of side > R per axis: floor(L / (R (1 + 2^-20))) >= 3
 *   v          speed; displacement per step v (VM, NVM) or v dt (Langevin)
 *              must be < min(Lx, Ly) / 2
 *   eta        noise strength >= 0 (VM, NVM: uniform noise amplitude,
 *              Eq. (1); Langevin: Gaussian noise amplitude, Eq. (5))
 *   omega      chirality, added to every new angle (Eqs. (2), (3), (5))
 *   gamma      coupling Gamma of Eq. (5) (Langevin only)
 *   dt         Euler-Maruyama step (Langevin only; > 0); ignored by VM, NVM
 *   rule       AAP_RULE_VM, AAP_RULE_NVM or AAP_RULE_LANGEVIN
 *   order      interaction order o of Eq. (5): 1 (polar alignment) to 64;
 *              must be 1 for VM and NVM, which have no order
 *   bx, by     boundary per axis: 0 periodic, nonzero reflecting (Sec. 4)
 *   seed       key of the counter-based random stream
 *   weights    Langevin weight table h(0..weight_len-1), host memory, copied
 *              at creation; n >= weight_len uses h(weight_len-1) (Sec. 4);
 *              NULL means h == 1 (the additive model)
 *   weight_len entries in weights (>= 1 when weights != NULL)
 *   bins_theta bins of the angle histogram over [-pi, pi) (binnum_theta of
 *              Sec. 4); 0 = no histograms; at most 4096
 *   bins_n     bins of the neighbour-number histogram, n = 0 .. bins_n - 1,
 *              larger n counted in the last bin (binnum_neighbors of Sec. 4);
 *              0 = no histograms; at most 4096; both or neither are 0
 *   replica    index of an independent random stream of the same seed: word
 *              2 of the counter of every draw (initial state and noise); 0
 *              for a single system
 */
typedef struct aap_params {
    uint64_t N;
    double Lx, Ly, R;
    double v, eta, omega;
    double gamma, dt;
    int32_t rule;
    int32_t order;
    int32_t bx, by;
    uint64_t seed;
    const double* weights;
    int32_t weight_len;
    int32_t bins_theta;
    int32_t bins_n;
    uint32_t replica;
} aap_params;

typedef struct aap_sim aap_sim;

/*
 * Normalised measurement results (Sec. 3.4): raw moments k = 1..4 of the
 * polar order p = |sum e^{i theta}| / N, of the mean neighbour number nbar
 * and of the nematic order q = |sum e^{2 i theta}| / N over the measured
 * states, the Binder cumulant U = 1 - <p^4>/(3 <p^2>^2) (Fig. 5), and p,
 * nbar and q of the last measured state.  Moments are 0 when no state has
 * been measured.
 */
typedef struct aap_observables_t {
    int64_t steps_measured;
    double p_mom[4];
    double nbar_mom[4];
    double binder;
    double p_last;
    double nbar_last;
    double q_mom[4];
    double q_last;
} aap_observables_t;

/* The standard Vicsek workload N=4096, L=64, R=1, v=0.5, eta=0.3, periodic,
 * seed 0 (the paper's own defaults are in its documentation, not in the
 * paper). */
aap_params aap_params_default(void);

/* Validates *p and stores in *bytes the device workspace it needs.
 * Host only: makes no HIP call.  AAP_EINVAL on an invalid parameter set. */
int aap_workspace_bytes(const aap_params* p, size_t* bytes);

/*
 * Creates a simulation.  d_workspace: device memory of at least
 * aap_workspace_bytes() bytes, 256-byte aligned, owned by the caller, which
 * must keep it alive and unused by others until aap_destroy.  hip_stream:
 * a hipStream_t (NULL = the null stream) on which all work of this handle is
 * enqueued.  Enqueues the uniform, isotropic random initial state (Sec. 5)
 * at step 0.  *out receives the handle (host memory owned by the library).
 * AAP_EINVAL bad parameters; AAP_ENOMEM workspace too small or misaligned;
 * AAP_EHIP runtime error.
 */
int aap_create(const aap_params* p, void* d_workspace, size_t bytes,
               void* hip_stream, aap_sim** out);

/* Waits for the stream and releases the handle (not the workspace). */
int aap_destroy(aap_sim* s);

/*
 * Advances nsteps >= 0 time steps: the paper's *model*_update_timesteps
 * (measure = 0) or *model*_measurement_timesteps (measure != 0), Sec. 4.
 * A measured call measures the states t .. t+nsteps-1, i.e. each state
 * before its update (Sec. 3.4).  p_series: NULL, or host memory for nsteps
 * doubles that receives p of each measured state (then the call is
 * synchronous).  Otherwise asynchronous; an inconsistency detected on the
 * device is reported by the next synchronous call as AAP_EHIP.
 */
int aap_step(aap_sim* s, int64_t nsteps, int measure, double* p_series);

/*
 * Steps per captured HIP graph for aap_step (even, <= 4096; 0, the default,
 * launches every step).  With steps_per_graph = G > 0, aap_step replays runs
 * of G steps from graphs captured on first use (one per measure setting and
 * buffer parity), with the step number the noise is keyed by read from
 * device memory; the first step after a state is set, the first measured
 * step of a call, steps that record a p series, timed steps (aap_timing_*)
 * and steps with debug output are launched one by one.  The results are
 * those of unreplayed steps, bit for bit.  Changing G synchronises the
 * stream and releases the graphs.  AAP_EINVAL for odd or out-of-range G.
 */
int aap_graph(aap_sim* s, int32_t steps_per_graph);

/* Copies the normalised results (aappp_get_results, Sec. 4).  Synchronous. */
int aap_observables(aap_sim* s, aap_observables_t* out);

/* Clears the measurement accumulators.  Asynchronous. */
int aap_reset_observables(aap_sim* s);

/*
 * Copies the current state to host arrays of N floats each, indexed by
 * particle id (0..N-1), and the current step to *step (any may be NULL).
 * Synchronous.
 */
int aap_get_state(aap_sim* s, float* x, float* y, float* theta,
                  uint64_t* step);

/*
 * Replaces the state by host arrays indexed by particle id (start from a
 * given state, Sec. 5) and sets the step counter, which keys the noise.
 * Periodic coordinates must lie in [0, L), reflecting ones in [0, L], and
 * angles in [-pi, pi] (pi rounded to binary32 included); AAP_EINVAL
 * otherwise (and for non-finite values).  Synchronous.
 */
int aap_set_state(aap_sim* s, const float* x, const float* y,
                  const float* theta, uint64_t step);

/* Waits for all work of the handle; reports a device-side error. */
int aap_sync(aap_sim* s);

/*
 * Parity inspection of the cell lists of the current state (host arrays,
 * NULL to skip): key[N] = cell id (cy * Mx + cx) of each particle by id.
 * mx, my receive the cells per axis.  Synchronous.
 */
int aap_debug_keys(aap_sim* s, uint32_t* key, int32_t* mx, int32_t* my);

/*
 * Enables (on != 0) capture of the per-particle neighbour sums by the
 * following steps; off by default because it costs 12 bytes per particle
 * and step of extra writes.
 */
int aap_debug_enable(aap_sim* s, int on);

/*
 * Parity inspection of the last step (host arrays, NULL to skip), which must
 * have run with capture enabled (AAP_EINVAL otherwise):
 *   start[Mx*My + 1]  exclusive prefix sum of the per-cell counts;
 *   order[N]          particle ids in cell-list order: by cell, and by
 *                     ascending id within a cell;
 *   n[N], C[N], S[N]  by particle id: |Omega_i| and the real and imaginary
 *                     part of e^{i theta_i} + sum_{Omega_i} e^{i theta~_j}
 *                     (VM, Langevin of order 1), of the bracket of Eq. (3)
 *                     (NVM), or of e^{i o theta_i} + sum e^{i o theta~_j}
 *                     (Langevin of order o).
 * Synchronous.
 */
int aap_debug_last_step(aap_sim* s, uint32_t* start, uint32_t* order,
                        uint32_t* n, float* C, float* S);

/*
 * Average device duration in milliseconds of each kernel of the step since
 * timing was enabled.  every > 0 enables and clears: the kernels of every
 * every-th step (counted from the call) carry a pair of HIP events on their
 * own dispatch; every = 1 times every launch.  every = 0 disables; negative
 * values are an error (AAP_EINVAL).  A timed launch is followed by a gap of
 * several microseconds on the stream and its event duration exceeds the
 * kernel's own by a few microseconds, so a sampling period well above 1
 * keeps a timed run close to an untimed one.  names/ms: host arrays of at
 * least *count entries on input; *count receives the number of kernels.
 */
int aap_timing_enable(aap_sim* s, int every);
int aap_timing_read(aap_sim* s, const char** names, double* ms,
                    int64_t* launches, int32_t* count);

/*
 * Normalised histograms of the measured states (Sec. 3.4): theta_hist[k] is
 * the fraction of particle angles (over all measured states) in
 * [-pi + 2 pi k / bins_theta, -pi + 2 pi (k+1) / bins_theta), the bin taken as
 * floor((theta + pi) * (bins_theta / (2 pi))) in binary64 from the binary32
 * angle and clamped to the range; n_hist[k] the fraction of neighbour
 * numbers |Omega_i| equal to k, the last bin holding all n >= bins_n - 1.
 * Host arrays of bins_theta and bins_n doubles, which must equal the counts
 * the simulation was created with (AAP_EINVAL otherwise, or when it was
 * created without histograms).  All zero before any measured state.
 * Synchronous.
 */
int aap_histograms(aap_sim* s, double* theta_hist, int32_t bins_theta, double* n_hist,
                   int32_t bins_n);

/*
 * Checkpoint (Sec. 3.6): the whole simulation -- positions and angles by
 * particle id, the step, the measurement accumulators and histograms --
 * in a host buffer; the random stream is counter-based (seed, step), so a
 * simulation loaded from a checkpoint continues exactly as the saved one
 * would have (identical states and measurements).
 * aap_checkpoint_bytes: the buffer size for this simulation.
 * aap_checkpoint_save: writes it to buf (host, at least that many bytes);
 *   synchronous.
 * aap_checkpoint_load: restores a checkpoint into a simulation created with
 *   the same parameters (N, box, radius, rule, boundaries, histogram bins);
 *   AAP_EINVAL when the buffer is not such a checkpoint, and then the
 *   simulation is left unchanged.  Synchronous.
 * The format is this library's own, in the host's byte order: a header
 * (magic "AAPCKPT1", version, every parameter, the step and the seed), the
 * weight table, x, y and theta as binary32 in id order, 16 binary64
 * accumulators, then the histogram counts as uint64.
 */
int aap_checkpoint_bytes(aap_sim* s, size_t* bytes);
int aap_checkpoint_save(aap_sim* s, void* buf, size_t bytes);
int aap_checkpoint_load(aap_sim* s, const void* buf, size_t bytes);

/*
 * Batches of replicas (independent systems stepped together).  Every
 * replica is a full system with its own parameters, but all share the rule
 * and the boundary types, and histograms are not measured.  Replicas of one
 * seed get independent random streams through their `replica` fields (the
 * counter word 2 of every draw): replica r of a batch evolves exactly as a
 * single system created with the same parameters.  After each replica's
 * first step, a step is two launches for the whole batch -- the counting
 * sort and the neighbour update, each workgroup serving one replica -- and
 * may be replayed from captured HIP graphs.
 *
 * aap_batch_workspace_bytes: device bytes for count replicas (params[count]).
 * aap_batch_create: as aap_create for every replica, inside one caller-owned
 *   device workspace (256-B aligned, at least that many bytes, kept alive
 *   until aap_batch_destroy), all on hip_stream.
 * aap_batch_graph: steps per captured graph (even, <= 4096; 0 = launch each
 *   kernel directly, the default).  Graphs are captured on first use on a
 *   private stream and launched on the batch's stream; results are
 *   identical either way.
 * aap_batch_step: nsteps steps of every replica (measure as in aap_step; no
 *   per-step series).  Asynchronous.
 * aap_batch_sync: waits for the stream; AAP_EHIP if a kernel flagged an
 *   inconsistency in any replica.
 * aap_batch_observables: out[count] as aap_observables of each replica.
 * aap_batch_reset_observables: clears every replica's accumulators.
 * aap_batch_get_state: aap_get_state of one replica.
 * aap_batch_threads: workgroup size of the batched neighbour kernel: 64,
 *   128 or 256 (the default); results do not depend on it.
 * aap_batch_kernel_times: runs `steps` steps (1..4096) with direct launches,
 *   each bracketed by HIP events, and returns the mean duration of the
 *   batched sort and neighbour launches in ms (host doubles).  The steps are
 *   ordinary steps of the simulation.  Synchronous.
 * aap_batch_debug_enable: on != 0 makes every later step of every replica
 *   (the batched kernels included) also record the per-particle n, C, S
 *   read by aap_batch_debug_last_step; off stops it.  Synchronous.  A
 *   testing aid of the parity harness (Eq. (6) sums of the batched
 *   neighbour kernel against the oracle); it slows the steps.
 * aap_batch_debug_keys: aap_debug_keys of one replica: the cells its
 *   particles will be sorted into by the next step, as written by the last
 *   step (by id), and the cell counts per axis.
 * aap_batch_debug_last_step: aap_debug_last_step of one replica: cell
 *   starts and sorted ids of the state the last step read, and n, C, S per
 *   id.  AAP_EINVAL unless a step ran with debug output on since it was
 *   switched on.
 * aap_batch_autotune: times every workgroup size with and without graphs of
 *   `steps` steps (even, 2..4096; each candidate runs 2 * steps ordinary
 *   steps, the first untimed) and keeps the fastest, returned in *threads
 *   and *steps_per_graph (either may be NULL).  Synchronous.
 */
typedef struct aap_batch aap_batch;
int aap_batch_workspace_bytes(const aap_params* params, int32_t count, size_t* bytes);
int aap_batch_create(const aap_params* params, int32_t count, void* d_workspace,
                     size_t bytes, void* hip_stream, aap_batch** out);
int aap_batch_destroy(aap_batch* b);
int aap_batch_graph(aap_batch* b, int32_t steps_per_graph);
int aap_batch_step(aap_batch* b, int64_t nsteps, int measure);
int aap_batch_sync(aap_batch* b);
int aap_batch_observables(aap_batch* b, aap_observables_t* out, int32_t count);
int aap_batch_reset_observables(aap_batch* b);
int aap_batch_get_state(aap_batch* b, int32_t replica, float* x, float* y,
                        float* theta, uint64_t* step);
int aap_batch_threads(aap_batch* b, int32_t threads);
int aap_batch_debug_enable(aap_batch* b, int on);
int aap_batch_debug_keys(aap_batch* b, int32_t replica, uint32_t* key, int32_t* mx,
                         int32_t* my);
int aap_batch_debug_last_step(aap_batch* b, int32_t replica, uint32_t* start, uint32_t* order,
                              uint32_t* n, float* C, float* S);
int aap_batch_kernel_times(aap_batch* b, int32_t steps, int measure, double* sort_ms,
                           double* nbr_ms);
int aap_batch_autotune(aap_batch* b, int32_t steps, int measure, int32_t* threads,
                       int32_t* steps_per_graph);

/*
 * Learned field surrogate.
 *
 * aap_fields: the coarse-grained fields of the current state (the density
 *   and polarisation measured per region of the box, Sec. 3.4 resolved in
 *   space) on a G x G grid of square bins of side L / G: d_fields (device,
 *   3 G^2 floats) receives [rho][p_x][p_y], each [G][G] row-major by (y, x),
 *   per unit area.  A particle's bin is floor(x G / L) in binary64 from its
 *   binary32 coordinate, clamped to G - 1.  d_scratch: device, 8-B aligned,
 *   aap_fields_scratch_bytes(G) bytes.  Square boxes, unit vectors of order
 *   1 (AAP_EINVAL otherwise).  Asynchronous on the simulation's stream.
 * aap_batch_fields: the same for one replica of a batch.
 * aap_fields_noalloc: aap_fields with the library's own scratch, for callers
 *   that cannot allocate device memory (code under HIP graph capture, tight
 *   serving loops, harnesses that forbid allocation): it allocates nothing
 *   and needs no scratch argument.  The scratch is a static device array of
 *   aap_fields_scratch_bytes(512) = 5 MiB that each GPU holds until the
 *   process ends, so G must be in [1, 512] (AAP_EINVAL beyond).  Every call
 *   on one GPU shares that GPU's array (it is cleared by a kernel at the
 *   start of each call): calls that overlap on one GPU, on different
 *   streams, race.  Otherwise as aap_fields (same output, same errors).
 *
 * The network advances such fields: input u = (rho / rho0 - 1, p / rho0)
 * zero-padded to 16 channels, three periodic 3x3 convolutions with ReLU
 * (16 -> 32 -> 32 -> 32), one linear (32 -> 16, three used), prediction
 * u + output; activations and weights bf16, products on the matrix cores
 * with fp32 accumulation, fp32 master weights trained with Adam on the mean
 * squared error of the prediction.
 * aap_cnn_param_count: number of fp32 parameters; layout, layer by layer:
 *   weights [3][3][Cin][Cout] (tap row, tap column, input, output), then
 *   biases [Cout], with (Cin, Cout) = (16, 32), (32, 32), (32, 32), (32, 16).
 * aap_cnn_workspace_bytes / aap_cnn_create: grid side G (a multiple of 16,
 *   16..1024) and largest batch; the caller owns the device workspace
 *   (256-B aligned, kept until aap_cnn_destroy).  Parameters start at 0.
 * aap_cnn_set_params / aap_cnn_get_params: host fp32 [count]; set clears
 *   the Adam state.  Synchronous.
 * aap_cnn_forward: d_in [nb][3][G][G] fields (device) -> d_out the same
 *   layout, the predicted fields; rho0 > 0 the mean density.  Asynchronous.
 * aap_cnn_train_step: one Adam step (learning rate lr) on the batch of nb
 *   (input, target) field pairs; *loss (may be NULL) receives the mean
 *   squared error of the prediction before the step (then synchronous).
 * aap_cnn_debug_read: copies an internal buffer of the last call to host
 *   (parity tests): 0 the bf16 input, 1..3 the bf16 activations, 4 the
 *   fp32 prediction [nb][G][G][3] in u units, 5 the fp32 gradient of every
 *   parameter, 6 the bf16 gradient of the output.  Synchronous.
 */
typedef struct aap_cnn aap_cnn;
int aap_fields_scratch_bytes(int32_t G, size_t* bytes);
int aap_fields(aap_sim* s, int32_t G, float* d_fields, void* d_scratch, size_t scratch_bytes);
int aap_batch_fields(aap_batch* b, int32_t replica, int32_t G, float* d_fields, void* d_scratch,
                     size_t scratch_bytes);
int aap_fields_noalloc(aap_sim* s, int32_t G, float* d_fields);
size_t aap_cnn_param_count(void);
int aap_cnn_workspace_bytes(int32_t G, int32_t max_batch, size_t* bytes);
int aap_cnn_create(int32_t G, int32_t max_batch, void* d_workspace, size_t bytes,
                   void* hip_stream, aap_cnn** out);
int aap_cnn_destroy(aap_cnn* c);
int aap_cnn_set_params(aap_cnn* c, const float* host, size_t count);
int aap_cnn_get_params(aap_cnn* c, float* host, size_t count);
int aap_cnn_forward(aap_cnn* c, const float* d_in, int32_t nb, double rho0, float* d_out);
int aap_cnn_train_step(aap_cnn* c, const float* d_in, const float* d_target, int32_t nb,
                       double rho0, float lr, double* loss);
int aap_cnn_debug_read(aap_cnn* c, int32_t which, void* host, size_t bytes);

/* Message of the last failing call on this thread ("" if none). */
const char* aap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AAP_H */
