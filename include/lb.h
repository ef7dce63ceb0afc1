/*
 * lb.h -- C ABI of the MI355X (gfx950) two-belt Shan-Chen lattice Boltzmann
 * library (liblb.so).
 *
 * The method is the one of Chibbaro, Falcucci, Chen, Shan, Chiatti, Succi,
 * "Lattice Boltzmann models for non-ideal fluids with arrested
 * phase-separation": a D2Q9 BGK lattice Boltzmann equation (eq. 1, section II)
 * on a periodic nx-by-ny lattice, driven by the two-belt pseudopotential force
 * of eq. (FORCE) (section III, Table 1) with psi(rho) = sqrt(rho0)
 * (1 - exp(-rho/rho0)), and monitored through the pseudo-potential energies
 * E_s, E_m and E_bulk of section V.
 *
 * One time step t -> t+1 at every site x:
 *   rho = sum_i f_i,  j = sum_i c_i f_i                        (section II)
 *   F   = -psi(x) sum_{k=1}^{24} K_k psi(x + c_k) c_k          (eq. FORCE)
 *         K_k = G1 w_k + G2 p(|c_k|^2) on the 8 first-belt links,
 *         K_k = G2 p(|c_k|^2) on the 16 second-belt links      (Table 1)
 *   u_eq = (j + tau F) / rho              (Shan-Chen velocity shift)
 *   f_i(x + c_i, t+1) = f_i - (f_i - f_i^eq(rho, u_eq)) / tau  (eq. 1)
 *
 * Conventions shared by every call:
 *   - Every function returns LB_OK (0) on success and a negative lb_status
 *     on failure; lb_last_error() then holds a message (per thread).
 *     Arguments are checked on the host before anything is launched, and a
 *     call that fails leaves the context unchanged.  The one exception is a
 *     HIP launch failure (LB_ERR_HIP) partway through a multi-step call
 *     (lb_step, lb_batch_step): launches issued before the failure cannot
 *     be withdrawn, so the context then holds the state they produce and
 *     lb_time reports the time level reached.  Nothing is thrown across
 *     this boundary.
 *   - Scalar fields are dense row-major double arrays of ny*nx values,
 *     site (x, y) at index y*nx + x.  Population arrays are dense
 *     [9][ny][nx] arrays of the storage type, population i in the D2Q9 order
 *     (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *   - Ownership: the caller owns every buffer it passes, including the
 *     device workspace, which the context borrows until lb_destroy.  The
 *     library owns only the small host-side context and allocates no device
 *     memory of its own.
 *   - Streams: a context issues all its work on the HIP stream given to
 *     lb_init (NULL = the null stream).  lb_step is asynchronous; calls that
 *     hand results to host memory synchronise the stream before returning.
 *     A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx lb_ctx;

/* Population storage.  LB_F64: double storage and arithmetic.  LB_F32:
 * float storage and arithmetic.  LB_F16DEV: half-precision storage of the
 * deviation f_i - w_i rho_ref, float arithmetic.  Global sums (mass and
 * energies) are accumulated in double for every storage. */
enum lb_storage { LB_F64 = 0, LB_F32 = 1, LB_F16DEV = 2 };

enum lb_status {
    LB_OK = 0,
    LB_ERR_INVALID = -1,   /* bad argument, sizes or parameters            */
    LB_ERR_HIP = -2,       /* HIP runtime error, or no usable device       */
    LB_ERR_NONFINITE = -3, /* a returned mass or energy is not finite      */
    LB_ERR_STATE = -4      /* unknown/destroyed context, full trace buffer */
};

typedef struct lb_params {
    int32_t nx, ny;      /* periodic lattice; each >= 5 so the +-2 links of the
                            second belt never alias onto one site; (nx+192)*ny < 2^31,
                            ny <= 65535                                           */
    int32_t storage;     /* lb_storage                                           */
    int32_t log_every;   /* > 0: record the section V energies every log_every
                            steps into the trace; 0: no trace                    */
    int32_t tile_x;      /* columns per workgroup: 0 (library choice), 64, 128
                            or 256                                               */
    int32_t tile_y;      /* rows per workgroup: 0 (library choice) or 1..4096    */
    int32_t tile_rows;   /* rows a workgroup updates per pipeline stage:
                            0 (library choice), 1 or 2                           */
    int32_t steps_per_launch; /* 0 (library choice: two per launch for LB_F32
                            and LB_F16DEV on large lattices), 1, or 2: with 2
                            the plain steps of LB_F32 and LB_F16DEV storage
                            between log points run two per launch (temporal
                            blocking); the fields are bit-identical to one
                            step per launch                                    */
    int64_t trace_cap;   /* rows the trace can hold (>= 0)                       */
    double tau;          /* BGK relaxation time, > 0.5 (the paper uses 1)        */
    double rho0;         /* psi scale, > 0 (the paper fixes rho0 = 1)            */
    double G1, G2;       /* first- and second-belt couplings, G < 0 attracts     */
    double rho_ref;      /* LB_F16DEV only: populations are stored as
                            f_i - w_i rho', rho' = rho_ref rounded to 20
                            significant bits so that the offsets and their
                            sum are exact in single precision (use the mean
                            initial density)                                    */
} lb_params;

/* Bytes of device workspace a context with these parameters needs, or 0 if
 * the parameters are invalid (host only; no device call). */
size_t lb_workspace_bytes(const lb_params* p);

/* LB_OK if the parameters are valid, LB_ERR_INVALID otherwise (host only). */
int lb_validate(const lb_params* p);

/* Resolved launch shape for these parameters: columns and rows per
 * workgroup, rows per pipeline stage and the workgroup count of the step
 * kernel (host only).  Any output may be NULL. */
int lb_launch_shape(const lb_params* p, int32_t* tile_x, int32_t* tile_y,
                    int32_t* tile_rows, int32_t* blocks);

/* Shape of the two-step launches for these parameters (host only): lanes
 * per workgroup (each workgroup produces tile_x - 6 columns), rows per
 * workgroup and workgroups; all three are 0 when plain steps run one per
 * launch.  Any output may be NULL. */
int lb_two_step_shape(const lb_params* p, int32_t* tile_x, int32_t* tile_y,
                      int32_t* blocks);

/* Create a context at t = 0 whose populations are the equilibrium
 * f_i^eq(rho_init, u_init) of section II (the paper starts from a fluid at
 * rest, section IV).
 *   workspace/bytes: device memory of at least lb_workspace_bytes(p) bytes,
 *       256-byte aligned, owned by the caller and borrowed until lb_destroy.
 *   rho_init: ny*nx densities, finite and > 0.
 *   ux_init, uy_init: ny*nx velocities or NULL for 0.
 *   inputs_on_device: 1 if the three input arrays are device pointers,
 *       0 if they are host memory (copied before lb_init returns).
 *   hip_stream: the hipStream_t all work of this context is issued on.
 * Errors: LB_ERR_INVALID (parameters, NULL pointers, short workspace,
 * non-finite or non-positive density), LB_ERR_HIP (no device, HIP error). */
int lb_init(lb_ctx** out, const lb_params* p, void* workspace, size_t bytes,
            const double* rho_init, const double* ux_init,
            const double* uy_init, int inputs_on_device, void* hip_stream);

/* Advance n >= 0 time steps of eq. (1) (t += n), asynchronously on the
 * context's stream.  With log_every > 0, the energies of every state
 * t' in [t, t+n) with t' % log_every == 0 that has not been recorded yet are
 * appended to the trace, computed by the step that leaves t' (the state at
 * t' is the pre-collision state, t' = 0 being the initial state); the state
 * reached at t+n is recorded by the next step or by lb_trace.  LB_ERR_STATE,
 * with nothing launched, if the trace cannot hold the new rows. */
int lb_step(lb_ctx* c, int64_t n);

/* Macroscopic fields of the state at the current t (section II):
 * rho = sum_i f_i and u = j / rho with j = sum_i c_i f_i.  Outputs are ny*nx
 * doubles each, device pointers if on_device = 1 (asynchronous), host
 * otherwise (synchronous).  Any output may be NULL to skip it. */
int lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, int on_device);

/* Section V observables of the state at the current t, synchronously:
 * out = {t, M = sum rho, E_s, E_m, sum psi^2, E_bulk = (G1+G2)/2 sum psi^2},
 * with E_s = 1/2 sum_x psi(x) sum_{i=0}^{8} (G1 w_i + G2 p_si) psi(x + c_i)
 * (rest weight p_s0 = 247/420 from eq. weights_1) and
 * E_m = 1/2 sum_x psi(x) sum_{i=1}^{16} G2 p_mi psi(x + c_mi).
 * Sums are in double, in an order fixed by the launch shape, so repeated
 * runs give bit-identical values.  LB_ERR_NONFINITE if any value is not
 * finite (out is still written). */
int lb_pseudo_energy(lb_ctx* c, double out[6]);

/* Copy up to cap trace rows (6 doubles each, same layout as
 * lb_pseudo_energy) into host memory; *n_rows receives the number of rows
 * recorded so far.  If the current t is a log point not recorded yet and the
 * trace has room, it is recorded first.  Synchronises the stream.
 * LB_ERR_NONFINITE if a copied row holds a non-finite value. */
int lb_trace(lb_ctx* c, double* out, int64_t cap, int64_t* n_rows);

/* Current time step t. */
int lb_time(lb_ctx* c, int64_t* t);

/* Export the pre-collision populations at t as a dense [9][ny][nx] array of
 * the storage type (for LB_F16DEV: the stored half deviations), to device
 * memory if on_device = 1 (asynchronous) or host memory (synchronous). */
int lb_get_state(lb_ctx* c, void* dst, int on_device);

/* Replace the state with populations in the lb_get_state layout and set the
 * time to t >= 0; the trace keeps its rows.  A lb_get_state / lb_set_state
 * round trip is exact. */
int lb_set_state(lb_ctx* c, const void* src, int on_device, int64_t t);

/* The link tables the kernels use, for the given couplings (host only):
 * cx, cy of the 24 links (first belt in D2Q9 order, then the second belt by
 * |c|^2 = 4, 5, 8, counter-clockwise from +x), K[k] their couplings, KE[0]
 * the rest coupling of E_s (G1 w_0 + G2 p_s0) and KE[1+k] = K[k]. */
int lb_tables(const lb_params* p, int8_t cx[24], int8_t cy[24], double K[24],
              double KE[25]);

/* Release the context (after synchronising its stream).  The workspace is
 * the caller's to free afterwards. */
int lb_destroy(lb_ctx* c);

/* Message describing the last failure on the calling thread. */
const char* lb_last_error(void);

/* ---------------------------------------------------------------------------
 * Batches: many independent periodic lattices, each with its own size,
 * couplings and initial density, advanced together by one kernel launch
 * per time step, or per two plain steps under the same rule as
 * lb_params.steps_per_launch (the step of every lattice is exactly the one
 * lb_step performs, so its fields are bit-identical to a lb_step run of the
 * same lattice).
 * ------------------------------------------------------------------------ */
typedef struct lb_batch lb_batch;

/* Workspace bytes for `count` lattices with parameters ps[0..count-1], or 0
 * if they are invalid.  All lattices must share storage, tile_x, tile_rows,
 * steps_per_launch, log_every and trace_cap (after the library's defaults
 * are applied); sizes, tile_y, tau, rho0, G1, G2 and rho_ref may differ. */
size_t lb_batch_workspace_bytes(const lb_params* ps, int32_t count);

/* Create a batch at t = 0; lattice i starts at rest with density
 * rho_init[i] (ny_i * nx_i doubles, host or device memory per
 * inputs_on_device).  Workspace and stream rules are those of lb_init.
 * When the stream is not the null stream, runs of plain steps are captured
 * into HIP graphs (one per run length and buffer parity) and replayed,
 * except for LB_F16DEV batches, whose rounding is seeded by the time level
 * a graph would freeze. */
int lb_batch_init(lb_batch** out, const lb_params* ps, int32_t count,
                  void* workspace, size_t bytes, const double* const* rho_init,
                  int inputs_on_device, void* hip_stream);

/* Advance every lattice n >= 0 steps, asynchronously.  With log_every > 0
 * the energies of each lattice are recorded at every log point in
 * [t, t+n], the state reached at t+n included, in each lattice's trace
 * (read with lb_trace on its member context).  LB_ERR_STATE, with nothing
 * launched, if the traces cannot hold the new rows. */
int lb_batch_step(lb_batch* b, int64_t n);

/* Turn graph capture of plain steps on or off (LB_ERR_INVALID to turn it
 * on for the null stream or for an LB_F16DEV batch). */
int lb_batch_use_graphs(lb_batch* b, int enable);

/* Launch shape of the batch's two-step launches: columns per workgroup
 * (each produces tile_x - 6 output columns), rows per workgroup and
 * workgroups per launch over all lattices; all three are 0 when the batch
 * runs one step per launch.  Any output may be NULL. */
int lb_batch_two_step_shape(lb_batch* b, int32_t* tile_x, int32_t* tile_y, int32_t* blocks);

/* Rows per workgroup of the batch's two-step launches: tile_y in [8, 64], or
 * 0 for the library's choice (the tallest of 48, 32, 24, 16 rows giving at
 * least 1400 workgroups).  Only the launch shape changes: fields stay
 * bit-identical.  Synchronises the stream and drops captured graphs.
 * LB_ERR_STATE if the batch runs one step per launch. */
int lb_batch_two_step_tile(lb_batch* b, int32_t tile_y);

/* Context of lattice i, owned by the batch: lb_moments, lb_pseudo_energy,
 * lb_trace, lb_time and lb_get_state accept it; lb_step, lb_set_state and
 * lb_destroy reject it with LB_ERR_STATE. */
int lb_batch_member(lb_batch* b, int32_t i, lb_ctx** member);

/* Release the batch and its member contexts (after synchronising). */
int lb_batch_destroy(lb_batch* b);

/* ---------------------------------------------------------------------------
 * Adjoint: gradients of a functional of the state after T steps of eq. (1)
 * from a fluid at rest (section IV start: f_i = w_i rho_init),
 *   L = (E(T) - E_target)^2 + beta * A(T),
 *   E = E_s + E_m (section V, as lb_pseudo_energy),
 *   A = sum_x sqrt(D_x rho^2 + D_y rho^2 + eps^2), D the central difference
 *       (x+1 minus x-1, halved): a measure of interface length,
 * with respect to G1, G2 and rho_init, by reverse-mode differentiation of
 * the discrete step (the transposed collision, force and streaming).  The
 * forward run keeps a copy of the populations every checkpoint_every steps;
 * the backward pass recomputes each segment from its copy, recording
 * (rho, j, psi) of every state, and steps the adjoint back through it.
 * Storage must be LB_F64 or LB_F32 (the arithmetic precision of both
 * passes; global sums in double); nx * ny <= 2^29 (LB_ERR_INVALID beyond);
 * log_every and trace_cap are ignored.
 * Workspace and stream rules are those of lb_init.
 * ------------------------------------------------------------------------ */
typedef struct lb_adj lb_adj;

typedef struct lb_adj_loss {
    double E_target;  /* E* of the energy term                              */
    double beta;      /* weight of the interface measure                     */
    double eps;       /* regularisation of |grad rho| in A, > 0              */
} lb_adj_loss;

/* Workspace bytes for T = nsteps >= 0 steps with a checkpoint every
 * checkpoint_every >= 1 steps (about ceil(T/every) population copies plus
 * two regions of `every` tape entries of 4 values per site: the backward
 * pass re-steps the next segment into one while it reads the other), or 0
 * if invalid.  With checkpoint_every >= T (one segment) the forward pass
 * tapes every step into a single region and the backward pass re-steps
 * nothing: the fastest backward pass, for 16 (FP32) or 32 (FP64) bytes per
 * site and step of workspace. */
size_t lb_adj_workspace_bytes(const lb_params* p, int64_t nsteps,
                              int32_t checkpoint_every);

/* Create an adjoint context.  p's tau, rho0, sizes, storage and launch
 * shape are used; G1 and G2 are given to each lb_adj_forward.  With a
 * stream (not the null stream) the context also creates a stream of its
 * own, at the default priority, for the backward pass's re-steps, which it
 * orders against hip_stream with events and destroys in lb_adj_destroy. */
int lb_adj_init(lb_adj** out, const lb_params* p, int64_t nsteps,
                int32_t checkpoint_every, void* workspace, size_t bytes,
                void* hip_stream);

/* Run T steps from f_i = w_i rho_init (ny*nx doubles, finite and > 0, host
 * or device memory per on_device) with couplings G1, G2 and evaluate the
 * loss: out = {L, E(T), A(T), M(T) = sum rho}.  Synchronous.
 * LB_ERR_NONFINITE if L or M is not finite. */
int lb_adj_forward(lb_adj* a, const double* rho_init, int on_device,
                   double G1, double G2, const lb_adj_loss* loss,
                   double out[4]);

/* Gradients of the loss of the last successful lb_adj_forward:
 * dG = {dL/dG1, dL/dG2} (host) and drho = dL/drho_init (ny*nx doubles, a
 * device pointer if on_device = 1, else host memory).  Synchronous; may be
 * called repeatedly.  LB_ERR_STATE without a successful forward. */
int lb_adj_backward(lb_adj* a, double dG[2], double* drho, int on_device);

/* Release the adjoint context (after synchronising its stream). */
int lb_adj_destroy(lb_adj* a);

/* ---------------------------------------------------------------------------
 * Structure factor (the Fourier analysis of section IV) of a density field
 * on an L x L periodic lattice, 5 <= L <= 2048:
 *   S(k) = (1/N) |sum_x (rho(x) - mean rho) exp(i k.x)|^2,
 *   k = (2 pi / L)(l, m), N = L^2;
 *   S_n = mean of S(k) over the shell (n - 1/2) <= |k| L / (2 pi) < n + 1/2,
 *         n = 0 .. nshell-1 (every mode lies in exactly one shell);
 *   kbar = sum_n n S_n / sum_n S_n (eq. rad, k in units of 2 pi / L);
 *   the droplet length scale is then R = L / (2 kbar) (k = 1 gives L/2).
 * Computed in double precision by FFTs in LDS (a direct transform when L is
 * not a power of two); every sum has a fixed order, so repeated calls give
 * bit-identical results.  Workspace and stream rules are those of lb_init.
 * ------------------------------------------------------------------------ */
typedef struct lb_sk lb_sk;

/* Number of shells of an L x L lattice (host only). */
int lb_sk_shells(int32_t L, int32_t* nshell);

/* Device workspace bytes for side L, or 0 if L is out of range. */
size_t lb_sk_workspace_bytes(int32_t L);

/* Create a structure-factor context for side L (builds the shell tables). */
int lb_sk_init(lb_sk** out, int32_t L, void* workspace, size_t bytes,
               void* hip_stream);

/* Structure factor of rho (L*L doubles, row-major [y][x], device memory if
 * on_device = 1, else host).  Writes, synchronously, up to cap shells:
 * shell[n] = S_n and counts[n] = modes in shell n (host arrays; either may
 * be NULL), *kbar (may be NULL) and, if spectrum is not NULL, the full S(k)
 * as a device array of L*L doubles indexed [m][l] (l, m the FFT indices of
 * x and y).  LB_ERR_NONFINITE if a shell value or kbar is not finite (kbar
 * is undefined for a uniform field). */
int lb_sk_compute(lb_sk* s, const double* rho, int on_device, double* shell,
                  int64_t* counts, int32_t cap, double* kbar, double* spectrum);

/* Release the context (after synchronising its stream). */
int lb_sk_destroy(lb_sk* s);

/* ---------------------------------------------------------------------------
 * Without allocation.
 * ------------------------------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of lb_pseudo_energy for a population array the caller holds,
 * with no context and no workspace.
 *   p: lattice size, storage, couplings and rho0 (and rho_ref for
 *      LB_F16DEV); the launch-shape fields are ignored.  The same limits as
 *      lb_validate apply; within them every lattice size is accepted.
 *   state: device pointer to the pre-collision populations as a dense
 *      [9][ny][nx] array of the storage type (the lb_get_state layout).
 *   t: the time level written to out[0].
 *   out: host memory, {t, M, E_s, E_m, sum psi^2, E_bulk} as in
 *      lb_pseudo_energy.  The sums are over the same site values in
 *      another fixed order.
 * Intermediate sums live in a fixed 32.8 KB device array of the library
 * (1024 partial rows of 4 doubles plus the result row) that each GPU holds
 * until the process ends; nothing is allocated, by the library or by HIP
 * on its behalf.  Every call on a GPU uses that one array, so calls that
 * overlap on one GPU (concurrent streams or threads) race: serialise them.
 * Synchronises hip_stream.  LB_ERR_NONFINITE if a value is not finite
 * (out is still written). */
int lb_pseudo_energy_state(const lb_params* p, const void* state, double t, double out[6],
                           void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
