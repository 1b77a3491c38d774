/*
 * rtn.h -- C ABI of the MI355X (gfx950) linearisation path of Real-time Neural MPC
 * (Salzmann et al., "Real-time Neural MPC: Deep Learning Model Predictive Control
 * for Quadrotors and Agile Robotic Platforms", RA-L 2023).
 *
 * What the library computes
 * -------------------------
 * Sec. IV-A: every SQP iteration needs, at every shooting node k of every MPC
 * instance, the continuity-condition parameters of the QP (eq. (2) and the
 * definitions below it):
 *     phi-bar_k = phi(x_k, u_k, f, dt),  A_k = d phi/d x_k,  B_k = d phi/d u_k,
 * where phi is one explicit RK4 step (Sec. III) of f = f_F + f_D: the nominal
 * quadrotor model f_F (eq. (6)) plus a learned residual network f_D (eq. (7)).
 * Real-time Neural MPC evaluates the network and its Jacobian once per node, as
 * one batch (Sec. IV-A), and forms phi, A_k and B_k with the network replaced by
 * its first-order local approximation f_D-bar + J_D [x - x_k; u - u_k] (eq. (4),
 * first order per Sec. IV-B).  rtn_linearize does exactly that on the GPU.
 * rtn_riccati solves the unconstrained LQ subproblem built from A_k, B_k (the
 * feedback phase, Sec. IV-B); rtn_train_step fits the residual network
 * (Sec. VII).
 *
 * Conventions for every function
 * ------------------------------
 *  - Return value is an rtn_status; RTN_OK (0) on success, a negative code
 *    otherwise, with a message available from rtn_last_error() (thread-local).
 *    Nothing aborts and no C++ exception crosses this interface.
 *  - All arguments are validated on the host before any work is enqueued.  On an
 *    error nothing has been enqueued and no output is guaranteed.
 *  - "device" pointers point to memory of the current HIP device; "host"
 *    pointers to ordinary CPU memory.  The caller owns every array argument and
 *    must keep device arrays alive until the stream has finished the call.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are stream-ordered and return before the GPU work completes, except where a
 *    function is documented as synchronous.
 *  - All arrays are row-major and node-major: node i of instance j is global
 *    node offsets[j] + i.  State x = [p(3), q(4) = (w,x,y,z), v(3), omega(3)]
 *    (13 floats), input u = rotor thrusts T_0..T_3 (4 floats), eq. (6).
 *  - A model may not be used from two streams at the same time (it owns
 *    workspace that calls share).
 */
#ifndef RTN_H
#define RTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rtn_status;
#define RTN_OK 0
#define RTN_EINVAL (-1)   /* invalid argument (message names it) */
#define RTN_ENOMEM (-2)   /* device or host allocation failed */
#define RTN_EHIP (-3)     /* a HIP runtime call failed (message holds its error string) */
#define RTN_ENOTSUP (-4)  /* valid request the library does not support (e.g. width) */

/* Arithmetic of the network part of a call.  RTN_FP32: fp32 matrix cores.
 * RTN_BF16: bfloat16 weights and activations, fp32 accumulation.
 * RTN_FP8: OCP FP8 E4M3 weights, activations and cotangents with static
 * per-tensor scales (see rtn_model_calibrate), fp32 accumulation.  In every mode
 * bias, activation, its derivative, f_D-bar, J_D and the RK4 chain are fp32. */
typedef enum { RTN_FP32 = 0, RTN_BF16 = 1, RTN_FP8 = 2 } rtn_precision;

/* Hidden-layer activation: SiLU a*logistic(a), or identity (linear network). */
typedef enum { RTN_ACT_SILU = 0, RTN_ACT_IDENTITY = 1 } rtn_activation;

/* Residual model variants (Sec. VI): the full residual of eq. (7) with input
 * [v, omega, q, u] and outputs [v-dot (world), omega-dot (body)], or the
 * simplified linear-acceleration residuals f_Da(v_B) and f_Da,u(v_B, u) whose
 * input is the body-frame velocity v_B = conj(q) (.) v (and u) and whose three
 * outputs add to v-dot; omega-dot gets no residual. */
typedef enum { RTN_INPUT_FULL = 0, RTN_INPUT_VB = 1, RTN_INPUT_VB_U = 2 } rtn_input;

/* Residual network descriptor (naming N-L-W of Sec. VII: L hidden layers of
 * width W).  (input, d_in, d_out) must be (RTN_INPUT_FULL, 14, 6),
 * (RTN_INPUT_VB, 3, 3) or (RTN_INPUT_VB_U, 7, 3); width one of 64, 128, 256,
 * 512, 1024; 1 <= n_hidden <= 16.  The variants support rtn_linearize and
 * calibration; training, rtn_linearize_exact and rtn_linearize_second return
 * RTN_ENOTSUP for them. */
typedef struct {
    int32_t d_in;
    int32_t d_out;
    int32_t n_hidden;
    int32_t width;
    int32_t activation; /* rtn_activation */
    int32_t input;      /* rtn_input */
} rtn_mlp_desc;

/* Quadrotor constants of eq. (6): mass [kg], diagonal inertia [kg m^2], arm =
 * centre-to-rotor distance of the X frame [m], c_tau = rotor reaction torque per
 * newton of thrust [m], g = gravity magnitude [m/s^2] (acting along -z world).
 * Rotor i sits at body (x,y) = arm/sqrt(2) * {(+,-), (-,-), (-,+), (+,+)}[i];
 * rotors 0 and 2 spin counter-clockwise, 1 and 3 clockwise (Fig. quad_model). */
typedef struct {
    float mass, Jx, Jy, Jz, arm, c_tau, g;
} rtn_quad;

typedef struct rtn_model rtn_model;

/* Library version string, static storage. */
const char* rtn_version(void);

/* Message of the last failing call on this thread ("" if none), valid until the
 * next failing call on the same thread. */
const char* rtn_last_error(void);

/* Number of float parameters of a network: for l = 1..L+1 the weight matrix
 * W_l [fan_out][fan_in] row-major (the convention y = W x + b) followed by the
 * bias b_l [fan_out].  This is the layout of every params_host buffer below. */
rtn_status rtn_param_count(const rtn_mlp_desc* desc, int64_t* count);

/* Create a model on the current device and copy the parameters (host, float,
 * rtn_param_count floats) into library-owned device memory.  The library
 * owns everything reachable from the model: fp32 master parameters, packed
 * bf16/fp8 copies, fp8 scales, gradients, Adam moments and workspace.
 * Synchronous.  *out is NULL on error. */
rtn_status rtn_model_create(const rtn_mlp_desc* desc, const float* params_host, rtn_model** out);

/* Free a model and everything it owns (synchronises the device first).  NULL is a no-op. */
rtn_status rtn_model_destroy(rtn_model* model);

/* Replace / read back the fp32 master parameters (host buffers, layout as
 * rtn_param_count).  Synchronous.  Setting parameters keeps the gradients and
 * Adam state and clears the fp8 calibration (its activation and cotangent
 * scales were measured on the old weights): RTN_FP8 calls fail with RTN_EINVAL
 * until rtn_model_calibrate runs again. */
rtn_status rtn_model_set_params(rtn_model* model, const float* params_host);
rtn_status rtn_model_get_params(rtn_model* model, float* params_host);

/* Static FP8 scales (the paper states no precision; the format and the scale
 * rule amax/448 are this library's choice).  Weight scales are amax(|W_l|)/448
 * and are refreshed whenever parameters change.  Activation and cotangent
 * scales are measured by running the network and its reverse sweep in fp32 over
 * n calibration nodes (device x [n][13], u [n][4]) and taking amax/448 per
 * tensor.  Synchronous.  RTN_FP8 calls on an uncalibrated model fail with
 * RTN_EINVAL, and every change of the parameters (rtn_model_set_params, an Adam
 * update of rtn_train_step or rtn_adam_step) returns the model to uncalibrated.
 * Finite operands beyond +-448 times their scale saturate; NaN stays NaN. */
rtn_status rtn_model_calibrate(rtn_model* model, int32_t n, const float* x, const float* u, void* stream);

/* Copy the scales to host: scales[0 .. 3L+2) = { weight scale of W_1..W_{L+1},
 * activation scale of z_0, h_1..h_L (L+1 values... index L+1..2L+1),
 * cotangent scale of layers L..1 (index 2L+2..3L+1) }.  *n_scales = 3L+2.
 * Values are 0 before calibration. */
rtn_status rtn_model_get_scales(const rtn_model* model, float* scales_host, int32_t* n_scales);

/* The hot path: continuity parameters of every node, eq. (2) with eq. (4).
 *   model      network f_D, or NULL for the nominal model alone (f_D = 0)
 *   prec       arithmetic of the network part (ignored when model is NULL)
 *   quad       host, quadrotor constants
 *   dt         RK4 step [s], > 0
 *   n_inst     number of MPC instances >= 1; offsets_host (host, int32
 *              [n_inst+1]) their node ranges: offsets[0] = 0, non-decreasing,
 *              offsets[n_inst] = n_nodes, each instance >= 1 node.  NULL means a
 *              single instance (n_inst must then be 1).  Nodes are independent,
 *              so offsets only describe the batch; they do not change results.
 *   n_nodes    total nodes >= 0 (0 is a valid empty call)
 *   x, u       device, fp32 [n][13], [n][4]: the iterate (x_k, u_k)
 * outputs (device, fp32):
 *   x_next     [n][13]      phi-bar_k
 *   A          [n][13][13]  A[k][i][j] = d x_{k+1,i} / d x_{k,j}
 *   B          [n][13][4]   B[k][i][j] = d x_{k+1,i} / d u_{k,j}
 *   f_D        nullable [n][6]      network output at the node (f_D-bar)
 *   J_D        nullable [n][6][14]  its Jacobian w.r.t. [v, omega, q, u]
 *              For the variants (RTN_INPUT_VB, RTN_INPUT_VB_U) both hold the
 *              network in the same embedded layout: outputs 0..2 are the
 *              v-dot residual and 3..5 zero; J_D columns 0..2 are d/d v_B,
 *              10..13 d/du (VB_U only), the rest zero.  The state Jacobian
 *              J_D dv_B/dx (through q and v) is formed inside the step.
 *   status     nullable uint8 [n]: 0 ok; bit0 non-finite network output or
 *              Jacobian; bit1 non-finite x_next, A or B.
 * The linearisation point (x_k, u_k, f_D-bar, J_D) is held fixed inside the RK4
 * step; A_k, B_k are the exact derivatives of that discrete map. */
rtn_status rtn_linearize(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                         int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                         const float* x, const float* u,
                         float* x_next, float* A, float* B,
                         float* f_D, float* J_D, uint8_t* status, void* stream);

/* The exact ("naive") linearisation of Sec. IV-A, for comparison with
 * rtn_linearize: the network and its Jacobian are evaluated at all four RK4
 * stage points (N*E function and N*E*2 derivative evaluations) instead of once
 * per node, and x_{k+1}, A_k, B_k are the exact derivatives of one RK4 step of
 * f_F + f_D.  Arguments, layouts and errors as rtn_linearize (model required;
 * no f_D / J_D / status outputs).  Uses model-owned workspace. */
rtn_status rtn_linearize_exact(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                               int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                               const float* x, const float* u, float* x_next, float* A, float* B,
                               void* stream);

/* The second-order local approximation of eq. (4): the network is replaced
 * inside the RK4 step by f_D-bar + J_D dz + 1/2 dz^T H_D dz (per output;
 * dz = z_0(x, u) - z_0(x_k, u_k), z_0 = [v, omega, q, u]) with (x_k, u_k,
 * f_D-bar, J_D, H_D) held fixed; x_{k+1}, A_k, B_k are the RK4 step and its exact
 * derivatives.  H_D (6 x 14 x 14 per node) is the network's Hessian by the chain
 * rule of second order.  prec must be RTN_FP32 (RTN_ENOTSUP otherwise); model
 * is required; arguments and layouts as rtn_linearize (no status output), plus
 *   H_D  nullable device fp32 [n][6][14][14]: H_D[k][j][a][b] = d^2 y_j / dz_a dz_b.
 * Nodes are processed in chunks of up to 4096 with stream-ordered scratch. */
rtn_status rtn_linearize_second(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                                int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                                const float* x, const float* u, float* x_next, float* A, float* B,
                                float* f_D, float* J_D, float* H_D, void* stream);

/* Feedback phase: backward Riccati recursion of the LQ problem
 *   min sum_k 1/2 [dx;du]^T blkdiag(Q,R) [dx;du] + q_k^T dx + r_k^T du
 *       + 1/2 dx_N^T Q_N dx_N + qN^T dx_N
 *   s.t. dx_{k+1} = A_k dx_k + B_k du_k + c_k          (eq. (2))
 * per instance, in fp64.  The optimal step is du_k = K_k dx_k + kff_k.
 *   offsets_host  as in rtn_linearize (NULL: one instance)
 *   A, B          device fp32 [n][13][13], [n][13][4] (promoted exactly)
 *   c             device fp64 nullable [n][13]: defects phi-bar_k - x_{k+1}
 *   Q_host, R_host, QN_host  host fp64 13x13, 4x4, 13x13 (symmetric; R + B^T P B
 *                 must be positive definite)
 *   q, r          device fp64 nullable [n][13], [n][4]; qN nullable [n_inst][13]
 * outputs (device fp64): K [n][4][13], kff [n][4], P nullable [n][13][13] = the
 * value-function Hessian P_k at node k (before the step at k is taken). */
rtn_status rtn_riccati(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                       const float* A, const float* B, const double* c,
                       const double* Q_host, const double* R_host, const double* QN_host,
                       const double* q, const double* r, const double* qN,
                       double* K, double* kff, double* P, void* stream);

/* rtn_riccati without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, outputs and results are those of rtn_riccati; the
 * cost matrices and instance offsets are staged in a fixed library-owned device
 * array (one per device, held until the process ends; about 260 KB) instead of
 * a stream-ordered allocation, so at most 65536 instances per call
 * (RTN_EINVAL beyond, nothing enqueued).  Calls that overlap on one device
 * (two host threads, or two streams running concurrently) race on that array;
 * calls on one stream are ordered.  The host arrays are consumed before the call
 * returns. */
rtn_status rtn_riccati_noalloc(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                               const float* A, const float* B, const double* c,
                               const double* Q_host, const double* R_host, const double* QN_host,
                               const double* q, const double* r, const double* qN,
                               double* K, double* kff, double* P, void* stream);

/* The same LQ problem with the input box of the QP (the input rows of eq. (3),
 * e.g. 0 <= u <= u_max written as du_lo = -u_k, du_hi = u_max - u_k):
 *   du_lo[k] <= du_k <= du_hi[k]  elementwise,
 * solved per instance by ADMM on the split du = z (z in the box): the Riccati
 * recursion of R + rho I is computed once, then each iteration is one backward
 * pass of the linear terms, one rollout from dx_0, an over-relaxed (1.6)
 * projection onto the box and a dual update, until max |du - z| < tol and
 * rho max |z - z_prev| < tol, or max_iter iterations.  Same A, B, c, Q, R, Q_N,
 * q, r, qN as rtn_riccati, plus
 *   dx0           device fp64 [n_inst][13]: initial deviation of each instance
 *   du_lo, du_hi  device fp64 [n][4] (du_lo <= du_hi required; the projection is
 *                 min(max(v, lo), hi))
 *   rho > 0, max_iter >= 1, tol > 0
 * outputs (device): du fp64 [n][4] (inside the box); dx nullable fp64 [n][13] and
 * dxN nullable fp64 [n_inst][13] rolled out with du; iters nullable int32
 * [n_inst]: iterations used (max_iter when not converged); resid nullable fp64
 * [n_inst][2]: primal and dual residual of the last iteration (an instance with
 * iters == max_iter and a residual above tol did not converge).  Scratch memory
 * is allocated and freed stream-ordered.  Errors as rtn_riccati. */
rtn_status rtn_riccati_box(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                           const float* A, const float* B, const double* c,
                           const double* Q_host, const double* R_host, const double* QN_host,
                           const double* q, const double* r, const double* qN,
                           const double* dx0, const double* du_lo, const double* du_hi,
                           double rho, int32_t max_iter, double tol,
                           double* du, double* dx, double* dxN, int32_t* iters, double* resid,
                           void* stream);

/* Forward pass of the LQ solution returned by rtn_riccati: the primal step of
 * the QP of Sec. IV-A (the step the feedback phase applies, Sec. IV-B).  Per
 * instance, from its initial deviation dx_0:
 *   du_k = K_k dx_k + kff_k,   dx_{k+1} = A_k dx_k + B_k du_k + c_k,  k = 0..N_i-1.
 *   offsets_host  as in rtn_linearize (NULL: one instance)
 *   A, B, c       as in rtn_riccati (c nullable)
 *   K, kff        device fp64 [n][4][13], [n][4] (from rtn_riccati)
 *   dx0           device fp64 [n_inst][13]
 * outputs (device fp64): du [n][4]; dx nullable [n][13] = dx_k at node k
 * (dx_0 repeated at the first node); dxN nullable [n_inst][13] = the terminal
 * deviation dx_{N_i}.  Errors: RTN_EINVAL on bad offsets or a missing required
 * pointer; nothing is enqueued then. */
rtn_status rtn_lq_rollout(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                          const float* A, const float* B, const double* c,
                          const double* K, const double* kff, const double* dx0,
                          double* dx, double* du, double* dxN, void* stream);

/* Network forward pass over a batch (device in [batch][14] -> out [batch][6]),
 * stashing what rtn_mlp_backward needs in the model: the residual network of
 * eq. (7) evaluated on training inputs (Sec. VII fits it offline to the
 * simulator's residual accelerations).  prec RTN_FP32 or RTN_BF16; the paper
 * states no precision, bf16 products with fp32 accumulation and fp32 master
 * weights are this library's choice. */
rtn_status rtn_mlp_forward(rtn_model* model, int32_t prec, int32_t batch,
                           const float* in, float* out, void* stream);

/* Backward pass of the last rtn_mlp_forward (same batch): given dL/dout
 * (device [batch][6]), ADD dL/dparams into the model's gradient buffer and, if
 * din is not NULL, write dL/din (device [batch][14]).  Exact backpropagation
 * through the network of eq. (7), in the precision of that forward pass. */
rtn_status rtn_mlp_backward(rtn_model* model, int32_t batch, const float* dout, float* din,
                            void* stream);

/* Zero the gradient buffer; copy it to host (rtn_param_count floats, synchronous). */
rtn_status rtn_model_zero_grad(rtn_model* model, void* stream);
rtn_status rtn_model_get_grad(rtn_model* model, float* grad_host);

/* One Adam step (bias-corrected, no weight decay) on the fp32 master parameters
 * from the gradient buffer; increments the model's step counter and refreshes
 * the packed copies. */
rtn_status rtn_adam_step(rtn_model* model, float lr, float beta1, float beta2, float eps,
                         void* stream);

/* Fused training step (Sec. VII): forward, loss = mean over (batch, 6) of
 * (net(in) - target)^2, backward, Adam.  in [batch][14], target [batch][6]
 * device fp32; loss (device fp32 scalar, nullable) receives the loss before the
 * update.  prec RTN_FP32 or RTN_BF16 (the matrix products; master weights and
 * Adam state are fp32). */
rtn_status rtn_train_step(rtn_model* model, int32_t prec, int32_t batch,
                          const float* in, const float* target,
                          float lr, float beta1, float beta2, float eps,
                          float* loss, void* stream);

/* Adam state to host: m and v (rtn_param_count floats each, nullable) and the step. */
rtn_status rtn_model_get_adam(rtn_model* model, float* m_host, float* v_host, int64_t* step);
rtn_status rtn_model_set_adam(rtn_model* model, const float* m_host, const float* v_host, int64_t step);

/* Autotuner of the network kernels.  For every (precision, width, depth,
 * size class = floor(log2 n_nodes)) the first rtn_linearize call times each
 * valid (tile variant, workgroup count) of the layer-chain forward and reverse
 * kernels on its own inputs -- and, for fp32 batches of at most 4096 nodes, the
 * small-batch path that launches one kernel per layer spread over many compute
 * units -- synchronising its stream while it does so, and keeps the fastest;
 * later calls, and the graphs captured from them, use the kept choice.  When
 * the stream is being captured by the caller the default shapes are used and
 * nothing is tuned.  RTN_TUNE=0 in the environment, or rtn_tune_mode(0), turns
 * tuning off (default shapes unless an entry exists); RTN_TUNE_FILE=path loads
 * a saved table before the first lookup and rewrites it after each new result.
 *   choice[5] = {path, forward variant, forward workgroups, reverse variant,
 *               reverse workgroups}: path 0 = layer-chain kernels, 1 = the
 *               small-batch path (fp32 only; the other entries are then unused);
 *               variant 0 is the default tile shape, 1 the alternative shape
 *               (widths 512 and 1024); workgroups 0 = two per compute unit
 *               (never more than there are row blocks).
 *   ms[2]     nullable: forward and reverse times measured when tuned.
 * rtn_tune_get: RTN_EINVAL when the key has no entry.  rtn_tune_set: RTN_EINVAL
 * when the choice names a path or shape that does not exist for the precision
 * and width.  The table is process-wide and guarded by a lock; save/load use a
 * text file. */
rtn_status rtn_tune_mode(int32_t on);
rtn_status rtn_tune_get(int32_t prec, int32_t width, int32_t n_hidden, int32_t n_nodes,
                        int32_t* choice, float* ms);
rtn_status rtn_tune_set(int32_t prec, int32_t width, int32_t n_hidden, int32_t n_nodes,
                        const int32_t* choice);
rtn_status rtn_tune_save(const char* path);
rtn_status rtn_tune_load(const char* path);

/* ---------------------------------------------------------------------------
 * Runtime workload of Sec. V: a double integrator x = [p, pdot], nominal
 * model f_F(x, u) = [pdot, u] (scalar input u), with a residual network f_D
 * from the state (2 values) to 2 values added to x-dot: n_hidden layers of
 * `width` units (the paper's runtime study sweeps two layers of 2..8192 units
 * and its Table II lists deeper ones; the 2-in / 2-out shape is the one its
 * parameter counts imply).  The paper sets the output layer to zero; any
 * weights work.
 *
 * Parameters (host fp32, flat): W_1 [width][2], b_1 [width], then for each
 * further hidden layer W_l [width][width], b_l [width], then W_out [2][width],
 * b_out [2].  1 <= n_hidden <= 64, 1 <= width <= 8192, activation as
 * rtn_activation.  The model keeps its own fp32 copy on the current device;
 * every call below runs on the device the model was created on.  Calls on one
 * model are not thread-safe (they share its workspace). */
typedef struct rtn_di_model rtn_di_model;

rtn_status rtn_di_param_count(int32_t n_hidden, int32_t width, int64_t* count);
rtn_status rtn_di_model_create(int32_t n_hidden, int32_t width, int32_t activation, const float* params_host,
                               rtn_di_model** out);
rtn_status rtn_di_model_destroy(rtn_di_model* model);

/* Preparation phase of Sec. IV-B for the double integrator: the network value
 * f_D-bar and Jacobian J_D at every node (by forward-mode tangents through the
 * layers), and one RK4 step (Sec. III) of f_F plus the first-order local
 * approximation eq. (4) held fixed, with its exact sensitivities (eq. (2)).
 *   model   nullable: NULL gives the nominal model alone (f_D = 0)
 *   dt      > 0;  n_nodes >= 0 (0 does nothing)
 *   x [n][2], u [n] (device fp32) -> x_next [n][2], A [n][2][2] (row-major,
 *   A[k][i][j] = d x_{k+1,i} / d x_{k,j}), B [n][2] = d x_{k+1} / d u_k;
 *   f_D [n][2], J_D [n][2][2] nullable (device fp32). */
rtn_status rtn_di_linearize(const rtn_di_model* model, float dt, int32_t n_nodes, const float* x, const float* u,
                            float* x_next, float* A, float* B, float* f_D, float* J_D, void* stream);

/* One real-time iteration (Sec. IV-B) of every instance: linearise at the
 * iterate, then solve the QP of Sec. IV-A (continuity eq. (2), no inequality
 * rows) with the Gauss-Newton tracking cost
 *   sum_k 1/2 |x_k - x_ref|_Q^2 + 1/2 R u_k^2 + 1/2 |x_N - x_ref|_QN^2
 * by the fp64 Riccati recursion and the rollout from dx_0 = x0 - x_0.
 *   model  nullable, as for rtn_di_linearize
 *   n_inst, offsets_host, n_nodes  as for rtn_linearize; every instance has at
 *          most 512 nodes
 *   Q_host [2][2], R_host [1], QN_host [2][2]  host fp64, finite, R > 0
 *   x [n][2], u [n]   iterate states x_0..x_{N-1} and inputs of each instance's
 *                     nodes (device fp32); xN [n_inst][2] terminal states;
 *                     x0 [n_inst][2] measured states; x_ref nullable
 *                     [n_inst][2] (zero when NULL)
 * outputs (device fp64): du [n], dx [n][2] (dx_0..dx_{N-1}), dxN [n_inst][2];
 *   gaps c_k = x_next_k - x_{k+1} (x_N for the last node).  A [n][2][2],
 *   B [n][2], x_next [n][2] nullable (device fp32): the linearisation used.
 * Widths <= 64 with at most 64 nodes per instance (and a NULL model) run as one
 * launch per call; wider networks or longer horizons, whose iteration is
 * several launches, replay a HIP graph captured for each argument set. */
rtn_status rtn_di_rti(const rtn_di_model* model, float dt, int32_t n_inst, const int32_t* offsets_host,
                      int32_t n_nodes, const double* Q_host, const double* R_host, const double* QN_host,
                      const float* x, const float* u, const float* xN, const float* x0, const float* x_ref,
                      double* du, double* dx, double* dxN, float* A, float* B, float* x_next, void* stream);

/* Kernel timing (tracing).  When enabled, every kernel the library launches is
 * bracketed by a pair of HIP events recorded on the call's stream (a few
 * microseconds of overhead per launch; leave it off for production timing).
 * rtn_profile_read waits for the recorded events, aggregates them per kernel
 * (name, number of launches, summed event time in milliseconds), writes up to
 * max_entries records to out (host, nullable), sets *n_entries to the number of
 * distinct kernels and clears the records.  Synchronous. */
typedef struct {
    char name[48];
    int32_t calls;
    double total_ms;
} rtn_kernel_time;

rtn_status rtn_profile_enable(int32_t on);
rtn_status rtn_profile_read(rtn_kernel_time* out, int32_t max_entries, int32_t* n_entries);

#ifdef __cplusplus
}
#endif

#endif /* RTN_H */
