/*
 * gpeps.h -- C ABI of the MI355X (gfx950) graph-PEPS simple-update library.
 *
 * The library evolves the kicked-Ising Trotter circuit of the paper (Model
 * section, Eq. 1-3): |psi(theta_h, n)> = U(theta_h)^n |0...0> with
 *   U = prod_<ij> RZZ_ij(theta_J) * prod_i RX_i(theta_h),
 *   RX(theta) = exp(-i theta X / 2), RZZ(theta) = exp(-i theta Z Z / 2)
 * (theta_J = -pi/2 is the exp(+i pi/4 Z Z) gate of Eq. 2), represented as a
 * graph PEPS (Method section: one tensor per qubit, one weight vector lambda
 * per edge, bond dimension chi = d_max) and evolved with the simple update:
 * for every RZZ gate the lambda weights of the neighbouring bonds are
 * absorbed, both site tensors are QR-reduced, the gate is contracted, a
 * truncated SVD restores bond dimension <= d_max and the weights are removed
 * again.  <Z_i> is read in the mean-field (lambda) environment (Method
 * section; Appendix B).  Around that loop: the inverse step U^dagger for
 * weight-N observables (Appendix B), belief-propagation gauging sweeps and the
 * BP readout (Results), and the hand-written adjoint of the whole evolution.
 *
 * Conventions shared by every call:
 *  - Every function returns gpeps_status; nothing throws, aborts or exits.
 *    On error, gpeps_last_error(ctx) describes it (for calls without a ctx,
 *    gpeps_last_error(NULL) returns the last such message of the thread).
 *  - Host pointers are plain CPU memory owned by the caller; they are read
 *    during the call only (or, for outputs, written before it returns).
 *  - Device pointers are HIP device memory on the current device.  The
 *    caller owns the workspace and the stream; the library allocates no
 *    device memory of its own.
 *  - All work is enqueued on the stream given to gpeps_init.  Calls that
 *    return data to the host synchronise that stream.
 *  - Qubits of a graph are 0..n_nodes-1; edges are given as vertex pairs.
 *    Within one Trotter layer, gates are applied colour class by colour
 *    class in ascending colour (the classes of a proper edge colouring act
 *    on disjoint qubit pairs), the order the paper leaves open.
 *  - Not thread-safe per context: calls on one ctx must be serialised.
 */
#ifndef GPEPS_H
#define GPEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPEPS_OK = 0,
  GPEPS_ERR_ARG = -1,        /* invalid argument (graph, sizes, config) */
  GPEPS_ERR_WORKSPACE = -2,  /* workspace missing or smaller than gpeps_workspace_size */
  GPEPS_ERR_HIP = -3,        /* a HIP runtime call failed; message holds hipGetErrorString */
  GPEPS_ERR_NUMERIC = -4,    /* device status word: NaN/Inf, zero two-site tensor, or Jacobi not converged */
  GPEPS_ERR_STATE = -5       /* call not valid in the current state (e.g. history full) */
} gpeps_status;

typedef enum {
  GPEPS_C64_F64SVD = 0,  /* site tensors complex64; QR, SVD, lambda and readout in float64 */
  GPEPS_C128 = 1         /* site tensors complex128; everything in float64 */
} gpeps_precision;

typedef enum {
  GPEPS_LAYER_RX = 0,   /* RX(theta_h) on every qubit of every instance */
  GPEPS_LAYER_RZZ = 1,  /* RZZ(theta_J) on every edge, colour class by colour class */
  GPEPS_STEP = 2,       /* one Trotter step: RX layer, RZZ layer, then <Z> readout into the history */
  GPEPS_STEP_INVERSE = 3, /* one application of U(theta_h)^dagger (Appendix B): RZZ(-theta_J) class by class
                           * in the forward order, then RX(-theta_h), then <Z> readout into the history */
  GPEPS_LAYER_REGAUGE = 4 /* one BP-gauging sweep: the simple update with the identity gate on every edge,
                           * class by class; nothing recorded (see gpeps_apply_layer) */
} gpeps_layer;

typedef enum {
  GPEPS_MODE_BATCHED = 0,  /* all (instance, edge) items of a colour class per launch; steps replayed as a hipGraph */
  GPEPS_MODE_PLAIN = 1     /* one edge of one instance per launch, no graph: the unbatched reference schedule */
} gpeps_mode;

/* One qubit graph.  edges: [n_edges][2] vertex ids (any order, no self-loops,
 * no duplicates); colour: [n_edges] proper edge colouring with values
 * 0..C-1, or NULL to let the library colour the edges (König/Kempe
 * alternating-path colouring in edge order; needs a bipartite graph).
 * Maximum degree 3. */
typedef struct {
  int32_t n_nodes;
  int32_t n_edges;
  const int32_t* edges;
  const int32_t* colour;
} gpeps_graph;

typedef struct {
  int32_t d_max;              /* bond dimension cap chi, 1..32 */
  int32_t precision;          /* gpeps_precision */
  double trunc_rel;           /* keep singular values s_k > trunc_rel * s_0 (and at most d_max of them) */
  int32_t max_jacobi_sweeps;  /* cap on one-sided Jacobi sweeps per SVD (<= 0: 40) */
  int32_t max_steps;          /* capacity of the per-step <Z> history (>= 1) */
  int32_t mode;               /* gpeps_mode */
  int32_t adjoint;            /* 1: store a checkpoint of the state at the start of every step and
                                 reserve the buffers of gpeps_backward, which recomputes each step;
                                 2: as 1, and the forward pass also keeps, for every step and colour
                                 class, the state before the class and the update's singular
                                 triplets, so gpeps_backward runs no recompute (workspace grows by
                                 max_steps x classes x (state + per-class buffers); steps are not
                                 replayed as a captured graph); 0: forward only */
} gpeps_config;

typedef struct gpeps_ctx gpeps_ctx;

/* Device workspace bytes needed for n_instances instances; instance k evolves
 * graphs[graph_of_instance[k]].  graphs: [n_graphs]; graph_of_instance:
 * [n_instances] host arrays.  Writes *bytes. */
gpeps_status gpeps_workspace_size(const gpeps_graph* graphs, int32_t n_graphs,
                                  const int32_t* graph_of_instance, int32_t n_instances,
                                  const gpeps_config* cfg, size_t* bytes);

/* Create a context over a caller-owned device workspace of ws_bytes bytes
 * (>= gpeps_workspace_size, 256-byte aligned) and a caller-owned HIP stream
 * (hipStream_t passed as void*; NULL = the default stream).  theta_h,
 * theta_j: [n_instances] host arrays of angles in radians (Eq. 2).  All host
 * inputs are copied.  The state is set to |0...0> (Eq. 3): every bond of
 * dimension 1 with lambda = 1.  On success *ctx owns host memory freed by
 * gpeps_destroy. */
gpeps_status gpeps_init(gpeps_ctx** ctx, const gpeps_graph* graphs, int32_t n_graphs,
                        const int32_t* graph_of_instance, int32_t n_instances,
                        const double* theta_h, const double* theta_j,
                        const gpeps_config* cfg, void* d_workspace, size_t ws_bytes,
                        void* hip_stream);

/* Return every instance to |0...0> and clear the history, the status word and the statistics. */
gpeps_status gpeps_reset(gpeps_ctx* ctx);

/* Enqueue `repeat` applications of a layer (gpeps_layer).  GPEPS_STEP is one
 * application of U(theta_h) (Eq. 2) followed by the <Z> readout stored as the
 * next row of the history; fails with GPEPS_ERR_STATE when the history
 * (cfg.max_steps rows) would overflow.  GPEPS_STEP_INVERSE is one application of
 * U(theta_h)^dagger with the current angles, recorded in the history the same way:
 * after n forward steps, gpeps_set_angles(pi/2, theta_J) and n inverse steps give
 * |omega(theta_h, n)> = U(pi/2)^{dagger n} |psi(theta_h, n)>, whose <Z_q> is the
 * expectation of the weight-N operator U(pi/2)^n Z_q U(pi/2)^{dagger n} (Appendix B).
 * GPEPS_LAYER_REGAUGE is one sweep of the simple update with the identity gate:
 * the state is unchanged up to singular values under cfg.trunc_rel, only its gauge
 * moves.  The fixed point of the sweeps is the fixed point of belief propagation
 * (Results: the simple update and BP share it), so k sweeps after each step are BP
 * gauging; at convergence the mean-field <Z> equals gpeps_bp_expect_z.
 * The adjoint covers forward steps only: with cfg.adjoint != 0, GPEPS_STEP_INVERSE,
 * GPEPS_LAYER_REGAUGE and the single layers GPEPS_LAYER_RX / GPEPS_LAYER_RZZ (which are not
 * checkpointed) fail with GPEPS_ERR_STATE.  Asynchronous: numeric faults are reported by the
 * next synchronising call. */
gpeps_status gpeps_apply_layer(gpeps_ctx* ctx, int32_t kind, int32_t repeat);

/* Mean-field <Z_v> of the current state for every qubit of every instance,
 * concatenated in instance order: out[sum_{k} n_nodes(graph_of_instance[k])]
 * float64.  out is device memory when out_on_device != 0 (then no
 * synchronisation), else host memory (synchronises and checks the status word). */
gpeps_status gpeps_expect_z(gpeps_ctx* ctx, double* out, int32_t out_on_device);

/* Belief propagation on the current state (Results: the simple update's lambda environment is
 * the fixed point of BP on the norm network <psi|psi>, and BP gauging does not improve on it).
 * Runs `iters` (0..100000) parallel BP iterations over every directed edge of every instance,
 * starting from trace-normalised identity messages, with the site tensors in the symmetric gauge
 * A_v = Gamma_v sqrt(lambda_e) on every leg; each new message is divided by its trace.  Then
 * writes the BP estimate of <Z_v> (every leg closed by its incoming message) for every qubit to
 * out ([total qubits] float64, device memory when out_on_device != 0, else host).  residual
 * (host, may be NULL) receives the largest Frobenius change of a message in the last iteration
 * (0 when iters = 0 or there are no edges).  The state and the <Z> history are not modified.
 * Synchronises unless out is on the device and residual is NULL. */
gpeps_status gpeps_bp_expect_z(gpeps_ctx* ctx, int32_t iters, double* out, int32_t out_on_device, double* residual);

/* gpeps_bp_expect_z for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the same iterations, readout,
 * outputs and errors, but the BP messages and the residual word live in a device array of the
 * library (64 MiB per GPU, held until the process ends) instead of the caller's workspace.
 * This call allocates nothing.  The messages need 4 * n_edges_total * d_max^2 * 16 bytes; more
 * than 64 MiB - 256 B returns GPEPS_ERR_ARG.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams or threads) race, and each call re-initialises the messages
 * and the residual word before use. */
gpeps_status gpeps_bp_expect_z_noalloc(gpeps_ctx* ctx, int32_t iters, double* out, int32_t out_on_device,
                                       double* residual);

/* Copy the per-step <Z> history recorded by GPEPS_STEP: out[steps_done][total
 * qubits] float64 (host or device as above).  *steps_done receives the row count. */
gpeps_status gpeps_z_history(gpeps_ctx* ctx, double* out, int32_t out_on_device, int32_t* steps_done);

/* Current bond dimension of every edge of every instance, in instance order:
 * out[sum_k n_edges(graph_of_instance[k])] int32 on the host.  Synchronises. */
gpeps_status gpeps_bond_dims(gpeps_ctx* ctx, int32_t* out);

/* Solver statistics accumulated since gpeps_init / gpeps_reset, written to
 * out[0..n-1] (host): 0 total one-sided Jacobi sweeps, 1 number of SVDs,
 * 2 largest sweep count of one SVD, 3 SVDs that hit max_jacobi_sweeps.
 * Entries past 3 are set to 0.  Synchronises the stream. */
gpeps_status gpeps_stats(gpeps_ctx* ctx, int64_t* out, int32_t n);

/* Replace the angles of every instance (theta_h, theta_j: [n_instances] host arrays, radians).
 * Later steps use the new angles; the state is not reset.  On a context with cfg.adjoint != 0
 * this fails with GPEPS_ERR_STATE once a step is recorded (the reverse sweep uses the current
 * angles for every recorded step): call gpeps_reset first.  Synchronises. */
gpeps_status gpeps_set_angles(gpeps_ctx* ctx, const double* theta_h, const double* theta_j);

/* Adjoint of the whole recorded evolution (the hand-written reverse sweep of the
 * simple update, with per-step checkpoints and recompute).  Needs cfg.adjoint = 1
 * and at least one GPEPS_STEP since the last reset.  The loss is
 * L = sum_v dl_dz[v] <Z_v>, the readout of the state after the last recorded step
 * (dl_dz: [total qubits] float64, device memory when dl_dz_on_device != 0, else host);
 * for the mean magnetisation of an instance dl_dz = 1/n_nodes on its qubits.
 * Writes dL/dtheta_h and dL/dtheta_J per instance into dtheta_h, dtheta_j
 * ([n_instances] host arrays; either may be NULL).  The truncation ranks of the
 * forward pass are held fixed.  The SVD backward broadens 1/(s_l^2 - s_k^2) as
 * d/(d^2 + 1e-12) / (s_l + s_k), d = s_l - s_k in units of the largest singular value
 * (the two-site tensor of each gate).  The forward state is left as it was.
 * Synchronises and checks the status word. */
gpeps_status gpeps_backward(gpeps_ctx* ctx, const double* dl_dz, int32_t dl_dz_on_device,
                            double* dtheta_h, double* dtheta_j);

/* Magnetisation (Fig. 2a): out[k] = mean of <Z_v> over the qubits of instance k in the last
 * recorded history row (the state after the last GPEPS_STEP / GPEPS_STEP_INVERSE), reduced on the
 * device in a fixed order.  out: [n_instances] float64, device memory when out_on_device != 0
 * (then no synchronisation), else host memory (synchronises and checks the status word).
 * GPEPS_ERR_STATE when no row has been recorded since the last reset. */
gpeps_status gpeps_mean_z(gpeps_ctx* ctx, double* out, int32_t out_on_device);

/* gpeps_backward for the magnetisation loss L = sum_k dl_dm[k] m_k, m_k as in gpeps_mean_z
 * (dl_dm: [n_instances] host array, finite values, GPEPS_ERR_ARG otherwise).  The seed
 * dL/d<Z_v> = dl_dm[k] / n_nodes(k) is formed on the device; everything else, the outputs and
 * the requirements (cfg.adjoint != 0, at least one GPEPS_STEP) are those of gpeps_backward. */
gpeps_status gpeps_backward_mean_z(gpeps_ctx* ctx, const double* dl_dm, double* dtheta_h, double* dtheta_j);

/* Wait for the stream and check the device status word. */
gpeps_status gpeps_sync(gpeps_ctx* ctx);

/* Kernel timing: enqueue `steps` Trotter steps (as GPEPS_STEP, so the history
 * advances) with the kernels launched one by one on the context stream and a
 * hipEvent recorded around every launch, then synchronise and write, for each
 * kernel kind k < n_kinds, the mean duration in milliseconds avg_ms[k] and
 * the number of launches n_launches[k].  Kinds: 0 RX layer, 1 lambda-absorb +
 * QR, 2 Theta + Jacobi SVD + truncation, 3 re-absorb, 4 <Z> readout.
 * kind_names (may be NULL) receives a static name per kind. */
gpeps_status gpeps_time_kernels(gpeps_ctx* ctx, int32_t steps, int32_t n_kinds, double* avg_ms,
                                int64_t* n_launches, const char** kind_names);

/* Kernel timing of the reverse sweep: gpeps_backward (dl_dz on the host; dtheta_h, dtheta_j as
 * there, either may be NULL) with a hipEvent recorded around every kernel launch, then for each
 * kind k < n_kinds the mean duration in milliseconds avg_ms[k] and the launch count
 * n_launches[k].  Kinds: 0 lambda-absorb + R factor, 1 Theta' + SVD keeping every singular
 * triplet, 2 re-absorb (these three are the recompute of each step when cfg.adjoint = 1; no
 * launches when cfg.adjoint = 2), 3 T-bar, 4 SVD / Theta' / QR backward, 5 site-tensor adjoints,
 * 6 RX adjoint, 7 readout seed, 8 lambda adjoints of the other legs (two launches per colour
 * class).  Every reduction of the reverse sweep runs in a fixed order, so dtheta_h and dtheta_j
 * are the same bits on every run.  kind_names (may be NULL)
 * receives a static name per kind.  Synchronises. */
gpeps_status gpeps_time_backward(gpeps_ctx* ctx, const double* dl_dz, double* dtheta_h, double* dtheta_j,
                                 int32_t n_kinds, double* avg_ms, int64_t* n_launches, const char** kind_names);

/* Tile shapes (the batching of the simple update, all edges of a colour class per launch):
 *   tiles[0]  rows per lane per Householder chunk of the QR reduction: 8 or 16 (complex128
 *             path; complex64 takes R from the Gram matrix and ignores it)
 *   tiles[1]  16-row tiles per wave of the complex64 re-absorb on the matrix cores: 1, 2, 4 or 8
 *             (ignored by the complex128 path)
 *   tiles[2]  threads per workgroup of the Theta' + SVD kernel when d_max <= 16: 64 (one wave
 *             per SVD, no workgroup barriers) or 256 (ignored for d_max > 16, which uses 256)
 * They change the blocking only; the complex64 re-absorb gives the same bits for every choice,
 * the Householder reduction and the SVD differ by float64 rounding.  Defaults 16, 2 and 256. */

/* Autotuner: run `steps` Trotter steps (1 <= steps <= cfg.max_steps) of the configured
 * workload once per candidate tile triple, timing every launch with hipEvents, keep for each
 * kernel the fastest candidate, then reset the state to the initial product state (as
 * gpeps_reset: the history is cleared).  tiles_out (may be NULL, else [3]) receives the choice.
 * The captured step graphs are rebuilt on the next GPEPS_STEP / GPEPS_STEP_INVERSE.  Synchronises. */
gpeps_status gpeps_autotune(gpeps_ctx* ctx, int32_t steps, int32_t* tiles_out);

/* Set the tiles explicitly (tiles[3], values as above; GPEPS_ERR_ARG otherwise).  Enqueued work keeps
 * the tiles it was launched with; the captured step graphs are rebuilt on the next GPEPS_STEP or
 * GPEPS_STEP_INVERSE.  On a context with cfg.adjoint != 0 this fails with GPEPS_ERR_STATE once a
 * step is recorded (the recompute of the reverse sweep must follow the forward blocking). */
gpeps_status gpeps_set_tiles(gpeps_ctx* ctx, const int32_t* tiles);

/* Destroy a context (device work already enqueued is synchronised first). */
gpeps_status gpeps_destroy(gpeps_ctx* ctx);

/* Message of the last failing call on ctx (or of the calling thread when ctx
 * is NULL).  Owned by the library, valid until the next call on ctx. */
const char* gpeps_last_error(const gpeps_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GPEPS_H */
