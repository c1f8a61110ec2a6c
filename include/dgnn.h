/*
 * dgnn.h -- C ABI of libdgnn.so: a nodal discontinuous Galerkin spectral
 * element (DGSEM) solver of the 3D compressible Navier-Stokes equations on
 * periodic hexahedral boxes, with a corrective-forcing neural network, for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is that of arXiv 2207.11571 ("Accelerating high order
 * discontinuous Galerkin solvers using neural networks: 3D compressible
 * Navier-Stokes equations"): a low-order DG operator p_LO plus a learned
 * forcing s (Eq. (4)), the forcing trained on s = G p_HO(q_HO) - p_LO(G q_HO)
 * (Eq. (5)), advanced with a three-stage third-order Runge-Kutta scheme.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: DG_OK (0) or a negative DG_E* code; dg_last_error() gives the
 *   text of the last failure on the calling thread.  No exception crosses the
 *   ABI.  Kernel execution errors surface at the next call or synchronisation.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Launch calls enqueue on it and return without synchronising unless stated.
 * Ownership: every device buffer (state, register, residual, workspace,
 *   weights, datasets, serving arena) is allocated by the caller and passed as
 *   a raw device pointer; the library never allocates per-solve device data.
 *   Opaque handles (dg_mesh, nn_model, solve_server) are host objects owned by
 *   the library and released with the matching *_free call.
 * Alignment: device buffers must be 256-byte aligned and must not alias each
 *   other unless stated.
 * State layout: q is double[5][E][n_p], E = N^3 elements, n_p = (P+1)^3 nodes,
 *   variables (rho, rho u, rho v, rho w, rho e); element e = ex + N (ey + N ez);
 *   node n = i + (P+1)(j + (P+1) k) with i along x; node (i, j, k) of element
 *   (ex, ey, ez) sits at x = ex h + (xi_i + 1) h / 2 (xi = Gauss-Legendre
 *   points), h = L / N, and likewise in y and z.
 */
#ifndef DGNN_H
#define DGNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DG_OK = 0,
    DG_EINVAL = -1,      /* null/aliased pointer, unsupported P or N, bad size     */
    DG_ENOSPC = -2,      /* workspace or arena too small                           */
    DG_EHIP = -3,        /* HIP runtime or launch error                            */
    DG_EAGAIN = -4,      /* solve_poll: not finished yet                           */
    DG_ENOENT = -5,      /* unknown request id                                     */
    DG_ENONFINITE = -6   /* NaN or Inf detected in a solve                         */
};

#define DG_MIN_ORDER 1
#define DG_MAX_ORDER 8

/* Copies the calling thread's last error text into buf (NUL-terminated). */
int dg_last_error(char* buf, size_t len);

/* ------------------------------------------------------------------ mesh */

/* Physical and discretisation parameters (Sec. 3.1 and App. A).
 * Nondimensionalisation: rho0 = V0 = 1, unit length, box side L (2 pi for the
 * Taylor-Green vortex), mu = 1/Re, T = p/rho, kappa = mu gamma/((gamma-1) Pr).
 * Cs > 0 switches on the Smagorinsky closure mu_t = rho (Cs h/(P+1))^2 |S|,
 * with turbulent Prandtl number Pr_t.  viscous = 0 gives the Euler equations.
 * p_ref is subtracted from the momentum fluxes (it changes the residual only
 * by rounding); pass p0 = 1/(gamma Mach^2). */
typedef struct dg_params {
    int32_t N;          /* elements per direction, 1..1024                     */
    int32_t P;          /* polynomial order, DG_MIN_ORDER..DG_MAX_ORDER          */
    int32_t viscous;    /* 1 Navier-Stokes (BR1), 0 Euler                       */
    int32_t reserved;
    double L;           /* box side                                              */
    double Re, Mach, gamma, Pr, Cs, Pr_t, p_ref;
} dg_params;

typedef struct dg_mesh dg_mesh;

/* Builds the Gauss-Legendre basis tables on the host, uploads them to the
 * current device and returns a mesh handle.  DG_EINVAL for an unsupported
 * P or N or a non-positive physical parameter. */
int dg_init_mesh(const dg_params* prm, dg_mesh** out);

/* Node count E n_p and the workspace bytes every dg_* call on this mesh
 * needs (face traces, interface fluxes, forcing and reduction buffers). */
int dg_mesh_query(const dg_mesh* m, int64_t* n_nodes, size_t* workspace_bytes);

void dg_free_mesh(dg_mesh* m);

/* Taylor-Green vortex initial condition, Eq. (11), written into q. */
int dg_init_tgv(const dg_mesh* m, double* q, void* stream);

/* dqdt = p(q): the weak-form DGSEM operator of Eq. (1)/(3) -- volume flux
 * divergence, Roe interface flux, BR1 gradients and viscous fluxes, optional
 * Smagorinsky closure.  No forcing.  q and dqdt must not alias. */
int dg_residual(const dg_mesh* m, const double* q, double* dqdt,
                void* ws, size_t ws_bytes, void* stream);

/* n_steps steps of the low-storage three-stage third-order Runge-Kutta
 * scheme (Sec. 3.1) of dq/dt = p(q) + s(q) (Eq. (4)), in place on q; k is
 * the Runge-Kutta register (same layout, contents on entry are ignored).
 * forcing == NULL advances the uncorrected low-order system (Eq. (3)); with a
 * model, s(q) is evaluated at every stage on the stage state. */
typedef struct nn_model nn_model;
int dg_rk_step(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps,
               const nn_model* forcing, void* ws, size_t ws_bytes, void* stream);

/* The low-order evolution of Algorithm 1: each of the n_steps steps is the
 * uncorrected Runge-Kutta step q^n -> q^{n+1} followed by the correction
 * q^{n+1} += dt s(q^n), s evaluated on the state at the start of the step
 * (forcing == NULL gives plain uncorrected steps).  The correction is added
 * in the last stage's update, so the face traces that the next step reads
 * already include it.  Arguments and errors as dg_rk_step. */
int dg_rk_step_post(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps,
                    const nn_model* forcing, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_rk_step
 * with the library's own scratch in place of the caller's workspace.  The
 * scratch is one static device array of DG_NOALLOC_SCRATCH_BYTES per GPU,
 * created when the code object loads and kept until the process ends; its
 * address is looked up once per device when the first mesh is built there.
 * The call allocates nothing (no hipMalloc / hipFree, no library allocator):
 * the caller passes q and k (same layout and meaning as dg_rk_step) and the
 * stream.  DG_ENOSPC when the mesh's workspace (dg_mesh_query) is larger
 * than DG_NOALLOC_SCRATCH_BYTES -- it holds 16^3 elements up to P = 3 and
 * 8^3 elements up to P = 8.  Every call on one GPU shares that GPU's array
 * (the last call's face traces, fluxes and forcing stay in it; nothing in it
 * needs to start at zero): calls that overlap on one GPU, from several
 * streams or threads, race and must be serialised by the caller.  Other
 * arguments and errors as dg_rk_step. */
#define DG_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int dg_rk_step_noalloc(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps,
                       const nn_model* forcing, void* stream);

/* Measurement twin of dg_rk_step: the same launches, each bracketed by a HIP
 * event pair on `stream`; out_ms (host, double[4]) receives the mean duration
 * in milliseconds of one launch of each stage kernel: [0] face traces,
 * [1] BR1 gradient pass, [2] network forcing (0 without a model),
 * [3] residual + stage update.  Where the BR1 pass and the network run as
 * one launch (P = 3 with a model reading all nodes of its variables, viscous,
 * E a multiple of 16) that launch is reported in [2] and [1] is 0.
 * Synchronises `stream`. */
int dg_profile_steps(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps,
                     const nn_model* forcing, void* ws, size_t ws_bytes, void* stream, double* out_ms);

/* Diagnostics, written to out_dev (device, double[8]):
 * [0] kinetic energy (volume mean of rho |v|^2 / 2), [1] max over nodes of
 * |v| + c, [2] min density, [3..7] integrals of the five conserved variables.
 * The reduction order is fixed: results are bitwise reproducible. */
int dg_diagnostics(const dg_mesh* m, const double* q, double* out_dev,
                   void* ws, size_t ws_bytes, void* stream);

/* Time step of Eq. (7) with the (P+1)^2 order scaling, from the state q:
 * min(CFL h/((P+1)^2 max(|v|+c)), CFL h^2/((P+1)^4 max(nu, gamma nu/Pr))),
 * nu = mu/min(rho).  Synchronises `stream`; *dt_host receives the value. */
int dg_stable_dt(const dg_mesh* m, const double* q, double cfl, double* dt_host,
                 void* ws, size_t ws_bytes, void* stream);

/* Infinity-norm error of Eq. (9) for rho u, rho v, rho w between q and q_ref
 * (same mesh): out_dev (device, double[3]). */
int dg_error_inf(const dg_mesh* m, const double* q, const double* q_ref, double* out_dev,
                 void* ws, size_t ws_bytes, void* stream);

/* The filter G of Sec. 2: nodal -> Legendre modal -> truncate -> nodal, per
 * element, from mesh src (order P_src) to mesh dst (same N, P_dst <= P_src).
 * Works on any 5-variable field (states and residuals alike). */
int dg_project(const dg_mesh* src, const dg_mesh* dst, const double* f_src, double* f_dst, void* stream);

/* Training pairs of Eq. (5) for one high-order snapshot q_hi:
 * x = G q_hi and y = G p_hi(q_hi) - p_lo(G q_hi), written as float rows
 * x_out[E][5 n_p_lo], y_out[E][5 n_p_lo] (row = element, variable-major).
 * ws must hold dg_forcing_target_ws() bytes. */
size_t dg_forcing_target_ws(const dg_mesh* hi, const dg_mesh* lo);
int dg_forcing_target(const dg_mesh* hi, const dg_mesh* lo, const double* q_hi,
                      float* x_out, float* y_out, void* ws, size_t ws_bytes, void* stream);

/* Training pairs of Algorithm 1 (the discrete increment over one low-order
 * step) for one low-order step of length dt_lo: with q_NN = G q_hi advanced
 * one uncorrected low-order Runge-Kutta step to q_NN', and q_hi advanced IN
 * PLACE over the same interval by m_sub >= 1 steps of dt_lo / m_sub (k_hi is
 * its Runge-Kutta register, contents ignored on entry),
 *   x = q_NN,   y = (G q_hi' - q_NN') / dt_lo,
 * written as float rows x_out[E][5 n_p_lo], y_out[E][5 n_p_lo].  Calling it
 * once per low-order step of a training window is the high-order evolution
 * of Algorithm 1.  ws must hold dg_increment_target_ws() bytes. */
size_t dg_increment_target_ws(const dg_mesh* hi, const dg_mesh* lo);
int dg_increment_target(const dg_mesh* hi, const dg_mesh* lo, double* q_hi, double* k_hi, double dt_lo,
                        int32_t m_sub, float* x_out, float* y_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------- forcing network */

/* The fully connected forcing network of Sec. 2.2, one network shared by all
 * elements: dims[0] = 5 n_p inputs (the element's state, variable-major),
 * hidden layers of dims[1..n_layers-1] units, dims[n_layers] = 5 n_p outputs.
 * Hidden activation: 0 = tanh, 1 = relu; the output layer is linear.
 * Parameters (caller-owned, device, float32) are packed layer by layer as
 * W_l[out][in] row-major followed by b_l[out].  The library keeps bfloat16
 * copies of the weights (w_bf16, caller-owned, nn_query's n_bf16 elements,
 * in the matrix cores' operand order, which the caller does not rely on)
 * for the matrix cores; biases stay float32.
 * norm (host, copied): mu_in[5], sigma_in[5], mu_out[5], sigma_out[5]:
 *   xhat = (x - mu_in[v]) / sigma_in[v],  s = mask[v] (sigma_out[v] yhat + mu_out[v]).
 * grad, adam_m, adam_v (device float32, n_params each) may be NULL for an
 * inference-only model; nn_init zeroes adam_m and adam_v. */
int nn_query(const int32_t* dims, int32_t n_layers, int64_t* n_params, int64_t* n_bf16);
int nn_init(const int32_t* dims, int32_t n_layers, int32_t activation,
            float* params, uint16_t* w_bf16, float* grad, float* adam_m, float* adam_v,
            const double* norm, const uint8_t* mask, void* stream, nn_model** out);
/* nn_init for a network that reads only the variables v with in_vars[v] != 0
 * and forces only those with out_vars[v] != 0 (host arrays of 5; NULL selects
 * all five), as the paper's network reads and forces the three momenta
 * (Sec. 2.2).  dims[0] = (variables read) x n_p and dims[n_layers] =
 * (variables forced) x n_p, the same n_p; input column j n_p + n is node n of
 * the j-th variable read, output columns likewise, and the forcing of the
 * other variables is zero.  norm and mask keep their five-variable layout.
 * nn_init is nn_init_io with every variable read and forced.  DG_EINVAL when
 * no variable is selected or the sizes do not fit the selection. */
int nn_init_io(const int32_t* dims, int32_t n_layers, int32_t activation,
               const uint8_t* in_vars, const uint8_t* out_vars,
               float* params, uint16_t* w_bf16, float* grad, float* adam_m, float* adam_v,
               const double* norm, const uint8_t* mask, void* stream, nn_model** out);
/* Re-derives the bfloat16 copies after the caller rewrote params. */
int nn_refresh(nn_model* model, void* stream);
/* Replaces the normalisation (host array of 20 doubles) and the mask. */
int nn_set_norm(nn_model* model, const double* norm, const uint8_t* mask);
/* Per-node normalisation, the paper's rescaling of the values at each node
 * (Sec. 2.2): col_dev (device, caller-owned, kept by reference until reset)
 * holds [4][5 n_p] doubles -- mu_in, sigma_in, mu_out, sigma_out of each
 * column v n_p + n of the five-variable element row -- and replaces the
 * per-variable maps of nn_init (the mask still applies).  NULL returns to
 * the per-variable maps.  DG_EINVAL when n_p does not fit the network. */
int nn_set_column_norm(nn_model* model, const double* col_dev, int32_t n_p);
void nn_free(nn_model* model);

/* dqdt += s(q) for every element of mesh m (bfloat16 matrix-core products,
 * float32 accumulation, float32 bias and activation, bfloat16 activations
 * between layers, float32 output, float64 forcing). */
int nn_forcing(const nn_model* model, const dg_mesh* m, const double* q, double* dqdt,
               void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of one nn_train_step with `batch` rows. */
size_t nn_train_ws(const nn_model* model, int32_t batch);

/* One Adam step (Kingma-Ba, bias-corrected, beta1 0.9, beta2 0.999, eps 1e-7)
 * of the MSE loss mean((yhat - (y - mu_out)/sigma_out)^2) (Sec. 2.1, Table 1:
 * mean square error) on a batch of training pairs: x, y are float32 rows of
 * all five variables, [.][5 n_p] variable-major, in physical units (device),
 * from which the network takes the variables it reads and forces; the loss
 * runs over the forced ones.  The batch is rows
 * idx[0..batch) of them (device int32, each < the caller's row count), or
 * rows 0..batch-1 when idx is NULL.  Forward and backward run on bfloat16
 * matrix cores with float32 accumulation; the float32 master weights, grad,
 * adam_m, adam_v are updated in place and the bfloat16 copies refreshed.
 * loss_dev (device float, may be NULL) receives the batch loss before the
 * update. */
int nn_train_step(nn_model* model, const float* x, const float* y, const int32_t* idx, int32_t batch,
                  float lr, float* loss_dev, void* ws, size_t ws_bytes, void* stream);

/* Per-variable mean and standard deviation of a training set (rows of
 * 5 n_p floats, variable-major): out_host receives mu_x[5], sigma_x[5],
 * mu_y[5], sigma_y[5], the layout nn_init's norm takes; each sigma is
 * floored at 1e-12 max(1, |mu|).  Two-pass float64 reduction on the device,
 * fixed order.  Synchronises `stream`; ws must hold nn_stats_ws(rows) bytes. */
size_t nn_stats_ws(int64_t rows);
/* Per-column mean and standard deviation of a training set (rows of 5 n_p
 * floats): out_dev (device) receives [4][5 n_p] doubles in nn_set_column_norm's
 * layout; each sigma floored at 1e-12 max(1, |mu|).  Two-pass float64
 * reduction, fixed order; ws must hold nn_column_stats_ws(rows, n_p) bytes. */
size_t nn_column_stats_ws(int64_t rows, int32_t n_p);
int nn_column_stats(const float* x, const float* y, int64_t rows, int32_t n_p, double* out_dev,
                    void* ws, size_t ws_bytes, void* stream);
int nn_data_stats(const float* x, const float* y, int64_t rows, int32_t n_p, double* out_host,
                  void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------- serving */

/* A continuous-batching server of Taylor-Green solves (one host thread and
 * one HIP stream of its own).  Solves are admitted by device footprint into
 * the caller's arena; the Runge-Kutta stages of all running solves of the
 * same order run in shared launches, so requests that arrive while others run
 * join them at the next step.  Each solve computes exactly what it would
 * compute alone (no cross-solve reductions).
 *
 * Fallback of the learned part: the uncorrected low-order evolution (Eq. (3),
 * the base method of Sec. 2.1) backs every corrected solve.  The server
 * checks a corrected solve's state after every round of steps and at each of
 * its kinetic-energy records: when a value is not finite, or the kinetic
 * energy exceeds (1 + 1e-3) times its initial value (the Taylor-Green flow
 * decays, so the forcing is driving it), the solve returns to the copy of
 * its state taken at the start of that round (already checked healthy),
 * drops the records after it and continues uncorrected to t_end.
 * solve_status reports fallback = 1 and the step it continued from; the
 * footprint of a corrected solve includes that state copy.  A non-finite
 * record of an uncorrected solve fails it with DG_ENONFINITE. */
typedef struct solve_server solve_server;

typedef struct solve_request {
    double Re, t_end, Mach, Cs;     /* Mach <= 0 means 0.1                         */
    int32_t P, N, use_nn;           /* use_nn requires model                       */
    int32_t ke_every;               /* record KE every ke_every steps (>= 1)       */
    const nn_model* model;
    double* ke_host;                /* host, ke_capacity doubles (t, KE) pairs; may be NULL */
    int32_t ke_capacity;            /* number of (t, KE) pairs ke_host holds       */
    int32_t nn_after_step;          /* use_nn: 0 forcing at every stage (Eq. (4)),
                                       1 correction after each step (Algorithm 1)  */
    double* q_out_host;             /* host, final state 5 E n_p doubles; may be NULL */
} solve_request;

enum { SOLVE_QUEUED = 0, SOLVE_RUNNING = 1, SOLVE_DONE = 2, SOLVE_FAILED = 3 };

typedef struct solve_status {
    int32_t state;                  /* SOLVE_*                                     */
    int32_t error;                  /* DG_* code when failed                       */
    int64_t steps, n_steps;         /* executed / total Runge-Kutta steps          */
    int32_t ke_count;               /* (t, KE) pairs written                       */
    int32_t fallback;               /* 1: a corrected solve continued uncorrected  */
    double t, dt;                   /* physical time reached, step size            */
    double latency_s;               /* completion - submission (done only)         */
    double queue_s;                 /* admission - submission                      */
    int64_t dof_updates;            /* E n_p x executed stages                     */
    int64_t fallback_step;          /* step it continued uncorrected from, or -1   */
} solve_status;

/* Bytes a solve of order P on N^3 elements occupies in the arena. */
size_t solve_footprint(int32_t P, int32_t N, int32_t use_nn);
int solve_server_create(void* arena, size_t arena_bytes, int32_t max_slots, solve_server** out);
/* Thread-safe and non-blocking.  DG_ENOSPC at once when the request can never
 * fit the arena; otherwise queued until a slot and arena space are free. */
int solve_submit(solve_server* srv, const solve_request* req, uint64_t* id);
/* Non-blocking: DG_OK with st filled when done or failed, DG_EAGAIN with st
 * filled while queued or running, DG_ENOENT for an unknown id. */
int solve_poll(solve_server* srv, uint64_t id, solve_status* st);
/* Blocks until no request is queued or running. */
int solve_server_drain(solve_server* srv);
/* Host-side test hook: on the next step boundary of request id, writes a NaN
 * into its state (exercises the non-finite detection of one solve). */
int solve_inject_nan(solve_server* srv, uint64_t id);
/* Totals: device-busy seconds (sum of step-batch wall times), launches. */
int solve_server_stats(solve_server* srv, double* busy_s, int64_t* batches);
void solve_server_free(solve_server* srv);

#ifdef __cplusplus
}
#endif
#endif
