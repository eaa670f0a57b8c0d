/*
 * lbmgnn.h — C ABI of the MI355X (gfx950) hot path of LBM-GNN
 * (Li, "LBM-GNN: Graph Neural Network Enhanced Lattice Boltzmann Method",
 * arXiv 2504.14494): the D2Q9 lattice Boltzmann step with the BGK collision
 * (Eq. 1, equilibrium Eq. 2) and the GNN-corrected collision (Eq. 3), plus the
 * hand-written backward pass and optimiser used to train the network (Eq. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller.  The
 *    library allocates no device memory; scratch space is passed in as
 *    `workspace` (size from lbm_workspace_bytes) and holds nothing between
 *    calls.  Calls whose work may run at the same time (other streams) need
 *    workspaces of their own: a call keeps partial sums and the fallback
 *    gate's counters there while its kernels run.  Host pointers appear only
 *    for small structs (lbm_tgv, lbm_fallback), which are read during the
 *    call.
 *  - Populations are stored shifted, g_i = f_i - w_i, as row-interleaved
 *    structure of arrays g[y][i][x]: lattice row y holds nine contiguous runs
 *    of nx values, one per direction i = 0..8 (x fastest; element
 *    (y*9 + i)*nx + x).  Batched arrays add a leading batch index:
 *    g[b][y][i][x].  The D2Q9 order is
 *    i = 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
 *        7:(-1,-1) 8:(1,-1),  w = 4/9, 1/9 (i = 1..4), 1/36 (i = 5..8).
 *  - All boundaries are periodic.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is only enqueued; no call synchronises the host.
 *  - Return value: 0 on success, a negative LBM_E* code on failure; then
 *    lbm_last_error() (thread-local) describes it.  Argument errors are
 *    reported before anything is enqueued.
 *  - Every kernel is deterministic: equal inputs give bitwise equal outputs
 *    (no floating-point atomics; reductions use a fixed order).
 *  - Only gfx950 devices are supported (LBM_EUNSUPPORTED otherwise).
 */
#ifndef LBMGNN_H
#define LBMGNN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,       /* bad argument, size or aliasing                 */
  LBM_EWORKSPACE = -2,   /* workspace / saved buffer too small             */
  LBM_EDEVICE = -3,      /* HIP runtime or launch error                    */
  LBM_EUNSUPPORTED = -4  /* current device is not gfx950                   */
};

/* Thread-local text of the last error ("" if none). */
const char *lbm_last_error(void);

/* ------------------------------------------------------------------------ *
 * Lattice Boltzmann, BGK                                                   *
 * ------------------------------------------------------------------------ */

/* Initial state at equilibrium (Eq. 2): g_i = f_i^eq(rho, u) - w_i at every
 * node, from caller fields rho, ux, uy [ny][nx].  Since the BGK collision
 * leaves f^eq unchanged this is also a valid post-collision state, which is
 * what lbm_step_* consume.  Requires nx, ny >= 1 and nx*ny < 2^31. */
int lbm_init(float *g, int nx, int ny, const float *rho, const float *ux,
             const float *uy, void *stream);
/* Same in FP64 (used to generate training targets on fine lattices). */
int lbm_init_f64(double *g, int nx, int ny, const double *rho,
                 const double *ux, const double *uy, void *stream);

/* Initial state on the slow manifold.  The pre-collision state is f^eq(rho, u)
 * plus the first-order Chapman-Enskog non-equilibrium
 * -(tau w_i rho / c_s^2) Q_i : S, with Q_i = e_i e_i - c_s^2 I and S the
 * symmetric velocity gradient taken by second-order central differences on
 * the periodic lattice (a textbook construction, not part of the paper's
 * method).  Like every state the steps consume, g holds its post-collision
 * image, f^eq - ((tau - 1) w_i rho / c_s^2) Q_i : S.  Unlike lbm_init it does
 * not excite the period-2 non-hydrodynamic mode, which at tau near 1/2 decays
 * only by |1 - 1/tau| per step.  Requires tau > 0. */
int lbm_init_ce(float *g, int nx, int ny, const float *rho, const float *ux, const float *uy,
                float tau, void *stream);
int lbm_init_ce_f64(double *g, int nx, int ny, const double *rho, const double *ux,
                    const double *uy, double tau, void *stream);

/* One time step of Eq. 1 in fused pull form.  g_src holds the post-collision
 * state of step t-1; the kernel gathers g_i(x) = g_src_i(x - e_i)
 * (streaming), forms rho and u, relaxes toward f^eq with omega = 1/tau and
 * writes the post-collision state of step t to g_dst.  g_src and g_dst must
 * not overlap (A/B buffers).  tau > 0.5 is expected but not enforced. */
int lbm_step_bgk(const float *g_src, float *g_dst, int nx, int ny, float tau,
                 void *stream);
/* Same in FP64. */
int lbm_step_bgk_f64(const double *g_src, double *g_dst, int nx, int ny,
                     double tau, void *stream);

/* Streaming alone, the left-hand side of Eq. 1 without the collision:
 * g_dst_i(x) = g_src_i(x - e_i), periodic, on `batch` lattices stored one
 * after another ([batch][ny][9][nx]).  Turns a post-collision state into the
 * next pre-collision state (e.g. to feed gnn_forward).  The buffers must not
 * overlap. */
int lbm_stream(const float *g_src, float *g_dst, int nx, int ny, int batch, void *stream);

/* Analytic decaying Taylor-Green field used for the error sums:
 * u_x = -u0 cos(kx X) sin(ky Y) D, u_y = u0 (kx/ky) sin(kx X) cos(ky Y) D,
 * X = x - x0, Y = y - y0, D = exp(-nu (kx^2 + ky^2) t). */
typedef struct lbm_tgv {
  double u0, kx, ky, x0, y0, nu, t;
} lbm_tgv;

/* Macroscopic fields and FP64 observables of a (post-collision) state: the
 * density and velocity moments of Eq. 2 (rho = sum f_i, rho u = sum e_i f_i)
 * and the quantities the Taylor-Green validation (validation section,
 * "Taylor-Green Vortex Validation") and the Reynolds-number study measure:
 * the L2 velocity error against the analytic decaying vortex and the kinetic
 * energy; plus the global mass and momentum the conservation checks and the
 * fallback gate use.
 * rho, ux, uy: [ny][nx] FP32 outputs, each may be NULL.
 * sums: NULL or device double[8] receiving
 *   [0] total mass  sum rho          [1] sum rho u_x    [2] sum rho u_y
 *   [3] kinetic energy 1/2 sum |u|^2
 *   [4] sum |u - u_a|^2   [5] sum |u_a|^2   (0 if analytic == NULL)
 *   [6] smallest population f_i      [7] number of f_i < 0
 * analytic: host pointer or NULL.  The sums are accumulated in FP64 from
 * per-node FP64 moments of the FP32 populations, in a fixed order.
 * workspace: >= lbm_workspace_bytes(LBM_WS_MOMENTS, 1, nx, ny, 0) bytes. */
int lbm_moments(const float *g, int nx, int ny, float *rho, float *ux,
                float *uy, const lbm_tgv *analytic, double *sums,
                void *workspace, size_t ws_bytes, void *stream);

/* Restriction of a fine FP64 run onto a coarse FP32 lattice: the training
 * pairs of Methodology, "Training Methodology" (coarse states regressed
 * toward high-resolution runs; the paper names no restriction, this is the
 * reading taken).
 * g_fine [nyf][9][nxf] FP64 shifted; if `pull` is set it is read through one
 * streaming step (a post-collision state becomes the next pre-collision one),
 * else it is taken as a pre-collision state.  Coarse node X sits on fine node
 * factor*X; its populations are f^eq(rho, u) of that fine node plus the
 * fine non-equilibrium momentum flux Pi^neq rebuilt as
 * w_i/(2 c_s^4) Q_i:Pi^neq scaled by factor*tau_c/tau_f.  If `unstream` is set
 * the coarse result is taken back through one coarse streaming step
 * (out_i(X) = R_i(X + e_i)), turning a pre-collision state of coarse step
 * m+1 into the post-collision state of step m.  nxf, nyf must be multiples of
 * factor.  Output g_coarse [nyf/factor][9][nxf/factor] FP32 shifted. */
int lbm_restrict(const double *g_fine, int nxf, int nyf, int factor,
                 double tau_f, double tau_c, int pull, int unstream,
                 float *g_coarse, void *stream);

/* One step of channel flow between two resting walls under a body force
 * (validation section, "Poiseuille Flow", Eq. 5), fused pull + forced
 * collision, same layout and shifted storage as lbm_step_bgk.  The paper
 * names no wall or forcing scheme; these are the textbook ones:
 *  - halfway bounce-back at y = -1/2 and y = ny - 1/2 (channel height ny):
 *    g_i(x, y) = src_i(x - cx_i, y - cy_i) when that row lies in the
 *    channel, else src_opp(i)(x, y); x is periodic;
 *  - body force rho * gx along x with Guo's forcing: u = (sum e_i f_i) / rho
 *    + gx / 2, f^eq at that u, plus (1 - 1/(2 tau)) w_i [3 (e_i - u)
 *    + 9 (e_i . u) e_i] . F.
 * tau must exceed 1/2.  The buffers must not overlap.  Steady state: the
 * parabola gx / (2 nu) (y + 1/2)(ny - y - 1/2), nu = (tau - 1/2) / 3, plus the
 * uniform bounce-back slip gx (16 (tau - 1/2)^2 - 3) / (24 nu). */
int lbm_step_channel(const float *g_src, float *g_dst, int nx, int ny, float tau,
                     float gx, void *stream);
int lbm_step_channel_f64(const double *g_src, double *g_dst, int nx, int ny,
                         double tau, double gx, void *stream);

/* x-averaged velocity profile of a channel state as lbm_step_channel leaves
 * it (post-collision populations f*, whose momentum includes the step's
 * force): prof[y] = mean over x of (sum_i e_ix f*_i) / rho - gx / 2, the
 * fluid velocity (sum_i e_ix f_i + F/2) / rho of the step; accumulated in
 * FP64 in a fixed order.  prof: device double[ny]. */
int lbm_channel_profile(const float *g, int nx, int ny, float gx, double *prof,
                        void *stream);

/* Plain copy of n floats (bandwidth reference for the BGK kernel). */
int lbm_copy(const float *src, float *dst, size_t n, void *stream);

/* VALU throughput reference for the corrected step (the GELU of "GNN
 * Architecture Details", tanh form): each of nblocks x 256
 * threads applies the network's GELU (tanh form, evaluated as
 * x / (1 + 2^(x (A + B x^2)))) `iters` times to eight independent register
 * values and writes their sum to out[thread].  `out` is a device array of
 * nblocks * 256 floats owned by the caller.  Rejects nblocks or iters outside
 * [1, 2^20] with LBM_EINVAL.  Time it on `stream` to obtain the GELU rate the
 * message-passing rounds are bound by: 8 * 256 * nblocks * iters GELUs. */
int gnn_gelu_rate(float *out, int nblocks, int iters, void *stream);

/* ------------------------------------------------------------------------ *
 * GNN-corrected collision (Eq. 3)                                          *
 * ------------------------------------------------------------------------ */

/* Parameter blob (FP32, row-major W[out][in]):
 *   W1[64][12] b1[64] W2[64][64] b2[64]                     encoder
 *   { We[64][130] be[64] Wn[64][128] bn[64] } x n_rounds    message passing
 *   Wh[10][64] bh[10]                                       head
 *   mu[12] sigma[12] s_delta                                constants
 * The first gnn_param_count(n_rounds) floats are trainable.  Features per
 * node are ((g_i)_{0..8}, rho - 1, u_x, u_y), normalised as (x - mu)/sigma.
 * Edge input is [h_receiver; h_sender; e_d] for the 8 neighbours
 * sender = receiver + e_d.  Activations are the tanh form of GELU.  The head
 * gives tau_adj = 0.5 + sigmoid(z_0) and the correction
 * delta f = s_delta * P z_{1..9}, P the orthogonal projector onto the null
 * space of the mass and momentum moments.  Weights and stored activations
 * are BF16 (round to nearest even) with FP32 accumulation; the head output
 * and the collision are FP32.  0 <= n_rounds <= 4 for the layout queries;
 * the message-passing entry points need n_rounds >= 1 (n_rounds = 0 is the
 * per-node network of lbm_step_simple). */
size_t gnn_param_count(int n_rounds);
size_t gnn_blob_len(int n_rounds);

/* Per-step fallback to plain BGK.  A step falls back when a post-collision
 * population is negative or not finite (bit 1) or when the relative change
 * of total mass against *mass is not <= drift_threshold (bit 2); the step's
 * output is then recomputed with the plain BGK collision from the same
 * source.  All pointers are device pointers:
 *   flags       OR-ed with the bits of this step (sticky; caller clears)
 *   n_fallback  incremented once per step that fell back (may be NULL)
 *   mass        FP64 total mass of the previous state; read, then replaced
 *               by the mass of this step's output.
 * A negative threshold forces the drift branch (used by tests). */
typedef struct lbm_fallback {
  double drift_threshold;
  unsigned *flags;
  unsigned *n_fallback;
  double *mass;
} lbm_fallback;

/* One time step with the GNN-corrected collision: pull streaming as in
 * lbm_step_bgk, then features, encoder, n_rounds rounds of message passing,
 * head, projection and Eq. 3, written to g_dst.  fb: host pointer or NULL
 * (no fallback gate).  workspace: >= lbm_workspace_bytes(LBM_WS_GNN_STEP,
 * 1, nx, ny, n_rounds) bytes.  params: device blob of gnn_blob_len floats. */
int lbm_step_gnn(const float *g_src, float *g_dst, int nx, int ny, float tau,
                 const float *params, int n_rounds, const lbm_fallback *fb,
                 void *workspace, size_t ws_bytes, void *stream);

/* lbm_step_gnn without a workspace and without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The step's scratch
 * (packed weights, the two node-state buffers, the gate's partials and
 * counters) lives in a static device array of the library, sized for at most
 * LBM_NOALLOC_MAX_NODES lattice nodes (about 16.6 MiB); each GPU the library
 * runs on holds its own copy until the process ends.  The first call on a
 * device looks up that device's copy; no call allocates or frees memory.
 * Every call on one GPU shares that GPU's copy: calls that may run at the
 * same time on one GPU (other streams, other host threads) race and must not
 * overlap.  Arguments, results and errors are those of lbm_step_gnn; in
 * addition nx * ny > LBM_NOALLOC_MAX_NODES is rejected with LBM_EINVAL
 * before anything is enqueued. */
#define LBM_NOALLOC_MAX_NODES 65536
int lbm_step_gnn_noalloc(const float *g_src, float *g_dst, int nx, int ny, float tau,
                         const float *params, int n_rounds, const lbm_fallback *fb,
                         void *stream);

/* The GNN-corrected collision alone (no streaming) on a batch of
 * independent periodic lattices: g_pre [batch][ny][9][nx] pre-collision,
 * g_post the corrected post-collision state, tau: device float[batch].
 * head_out: NULL or [batch][ny][nx][10] FP32 head outputs z.
 * saved: NULL for inference, or >= lbm_workspace_bytes(LBM_WS_GNN_SAVED, ...)
 * bytes that receive the activations gnn_backward needs.
 * workspace: >= lbm_workspace_bytes(LBM_WS_GNN_FORWARD, ...) bytes. */
int gnn_forward(const float *g_pre, float *g_post, int batch, int nx, int ny,
                const float *tau, const float *params, int n_rounds,
                float *head_out, void *saved, size_t saved_bytes,
                void *workspace, size_t ws_bytes, void *stream);

/* Backward pass of the training step (Methodology, "Training Methodology":
 * supervised regression of the corrected collision, loss Eq. 4).
 * Gradient of a scalar loss with respect to the trainable parameters, given
 * dL_dgpost = dL/d g_post at the output of the forward call that filled
 * `saved` (same g_pre, tau and params): gnn_forward for n_rounds >= 1 (GELU
 * message-passing network), simple_forward for n_rounds = 0 (the per-node
 * ReLU network of Fig. 2).  BF16 rounding of the forward is treated as the
 * identity.  grad: device float[gnn_param_count(n_rounds)],
 * overwritten.  workspace: >= lbm_workspace_bytes(LBM_WS_GNN_BACKWARD, ...). */
int gnn_backward(const float *dL_dgpost, const float *g_pre, const void *saved,
                 int batch, int nx, int ny, const float *tau,
                 const float *params, int n_rounds, float *grad,
                 void *workspace, size_t ws_bytes, void *stream);

/* The per-node corrected collision of the paper's Fig. 2 network: the same
 * features, a 12 -> 64 -> 64 MLP with ReLU and the 64 -> 10 head (tau_adj,
 * projected delta f, Eq. 3), with no message passing, fused into the pull
 * step (one read and one write of the nine populations per node).  params:
 * device blob of gnn_blob_len(0) floats (the zero-round layout above).
 * workspace: >= lbm_workspace_bytes(LBM_WS_SIMPLE, ...) bytes.  fb as for
 * lbm_step_gnn (NULL = no gate). */
int lbm_step_simple(const float *g_src, float *g_dst, int nx, int ny, float tau,
                    const float *params, const lbm_fallback *fb, void *workspace,
                    size_t ws_bytes, void *stream);
/* lbm_step_simple on the channel of lbm_step_channel (validation section,
 * "Poiseuille Flow"): halfway bounce-back walls below row 0 and above row
 * ny - 1, x periodic, body force rho * gx along x.  The network reads Guo's
 * velocity u = (sum e f + F / 2) / rho among its features, f^eq is taken at
 * that velocity, and Guo's source is added at the network's effective
 * relaxation time tau * tau_adj (the paper names no forcing scheme for its
 * network).  The fallback, when fb is given, is the forced BGK channel step
 * of lbm_step_channel.  gx must be finite (LBM_EINVAL otherwise); other
 * arguments and errors as for lbm_step_simple. */
int lbm_step_simple_channel(const float *g_src, float *g_dst, int nx, int ny,
                            float tau, float gx, const float *params,
                            const lbm_fallback *fb, void *workspace,
                            size_t ws_bytes, void *stream);
/* The same collision alone (no streaming) on a batch of pre-collision states
 * [batch][ny][9][nx], tau: device float[batch]; head_out NULL or
 * [batch][ny][nx][10].  saved: NULL for inference, else a device buffer of
 * >= lbm_workspace_bytes(LBM_WS_GNN_SAVED, batch, nx, ny, 0) bytes that
 * receives what gnn_backward (n_rounds = 0) needs: the BF16 features, both
 * hidden layers (fragment order) and the FP32 head outputs per node. */
int simple_forward(const float *g_pre, float *g_post, int batch, int nx, int ny,
                   const float *tau, const float *params, float *head_out,
                   void *saved, size_t saved_bytes, void *workspace,
                   size_t ws_bytes, void *stream);

/* Eq. 4 with N = batch*nx*ny nodes: loss = scale/N * sum (a - b)^2 over all
 * nodes and the 9 populations, accumulated in FP64 into *loss (device
 * double); grad_a (NULL or like a) receives d loss / d a in FP32.
 * workspace: >= lbm_workspace_bytes(LBM_WS_MSE, batch, nx, ny, 0) bytes. */
int gnn_mse(const float *a, const float *b, int batch, int nx, int ny,
            double scale, double *loss, float *grad_a, void *workspace,
            size_t ws_bytes, void *stream);

/* Eq. 4 with the per-node residual r = a - b (nine populations) weighted by
 * a symmetric 9 x 9 matrix Q: loss = scale/N * sum over nodes of r^T Q r,
 * grad_a = 2 scale/N * Q r.  Q = identity is gnn_mse; Q = M^T W M with M a
 * moment basis of D2Q9 and W diagonal weights the residual's moments (a
 * training option beside the paper's plain Eq. 4, used to weight the
 * hydrodynamic moments over the non-hydrodynamic ones).  a, b, grad_a in the
 * row-interleaved layout [batch][ny][9][nx]; q: host, 81 doubles, row-major,
 * must be finite and symmetric (LBM_EINVAL otherwise); products with Q in
 * FP64.  workspace: >= lbm_workspace_bytes(LBM_WS_MSE, batch, nx, ny, 0). */
int gnn_mse_weighted(const float *a, const float *b, int batch, int nx, int ny,
                     const double *q, double scale, double *loss, float *grad_a,
                     void *workspace, size_t ws_bytes, void *stream);

/* One optimiser step of the training loop (Methodology, "Training
 * Methodology"; the paper names no optimiser: Adam, Kingma and Ba, Algorithm
 * 1) on n FP32 parameters with FP32 moments m, v
 * (zero before the first step); step is the 1-based count after this one. */
int gnn_adam(float *params, const float *grad, float *m, float *v, size_t n,
             float lr, float beta1, float beta2, float eps, int step,
             void *stream);

/* ------------------------------------------------------------------------ *
 * Workspace sizes                                                          *
 * ------------------------------------------------------------------------ */
enum {
  LBM_WS_MOMENTS = 0,
  LBM_WS_GNN_STEP = 1,
  LBM_WS_GNN_FORWARD = 2,
  LBM_WS_GNN_SAVED = 3,
  LBM_WS_GNN_BACKWARD = 4,
  LBM_WS_MSE = 5,
  LBM_WS_SIMPLE = 6
};
/* Bytes needed by operation `op` for the given sizes (0 if op is unknown). */
size_t lbm_workspace_bytes(int op, int batch, int nx, int ny, int n_rounds);

#ifdef __cplusplus
}
#endif

#endif /* LBMGNN_H */
