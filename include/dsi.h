/*
 * dsi.h -- C ABI of libdsi, a single-GPU (MI355X, gfx950) implementation of the
 * DeepInverse recovery path (Mousavi & Baraniuk, "Learning to Invert: Signal
 * Recovery via Deep Convolutional Networks", arXiv 1701.03891).
 *
 * The path, as the paper defines it:
 *   - measurement  y = Phi x, Phi an M x N matrix, M << N            (Sec. 1)
 *   - proxy        x~ = Phi^T y, a fixed fully connected layer,
 *                  read as an n1 x n2 image (n1 n2 = N)                 (Sec. 4)
 *   - L conv layers, each S(ReLU(W * a + b)) with zero padding and a
 *                  crop S back to n1 x n2; 1 -> 64 -> 32 -> 1 channels,
 *                  11 x 11 filters in the paper's experiments          (Sec. 4 Eq. 1, Sec. 5)
 *   - training     L(Omega) = (1/l) sum_i ||M(y_i, Omega) - x_i||^2,
 *                  minimised by backpropagation                        (Sec. 4)
 *
 * Conventions shared by every call:
 *   - Tensor pointers are DEVICE pointers, allocated and owned by the caller,
 *     unless a comment says "host".  The library never frees or reallocates
 *     caller memory.  Device buffers must be 16-byte aligned.
 *   - Images are row-major: pixel p = i*n2 + j.  Batches are outermost.
 *   - "*" in Eq. (1) is taken as 2-D cross-correlation; the crop S of the full
 *     correlation is the centred "same" output with zero padding (k-1)/2.
 *   - Work is enqueued on the caller's HIP stream (`stream`, a hipStream_t;
 *     NULL is the default stream).  No call synchronises the device except
 *     where stated; errors from kernels that already ran surface as DSI_E_HIP
 *     on a later call.
 *   - Every call returns a dsi_status.  Argument errors are detected before
 *     any launch and leave every output untouched; dsi_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - One dsi_ctx per host thread, or external locking.  Calls on one ctx that
 *     share its workspace must be ordered on one stream.
 */
#ifndef DSI_H
#define DSI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSI_OK = 0,
  DSI_E_NULL = 1,   /* a required pointer is NULL */
  DSI_E_SHAPE = 2,  /* a size is out of range or inconsistent */
  DSI_E_DTYPE = 3,  /* unsupported precision for this network */
  DSI_E_ALIGN = 4,  /* a device pointer is not 16-byte aligned */
  DSI_E_NOMEM = 5,  /* device allocation failed */
  DSI_E_HIP = 6,    /* a HIP runtime call or an earlier kernel failed */
  DSI_E_STATE = 7   /* object used in a state that does not allow the call */
} dsi_status;

typedef enum {
  DSI_F32 = 0,      /* FP32 operands, FP32 accumulation */
  DSI_BF16 = 1,     /* BF16 operands (round to nearest even), FP32 accumulation */
  DSI_FP8_E4M3 = 2, /* OCP FP8 e4m3 operands with power-of-two per-tensor scales, FP32 accumulation */
  DSI_F64 = 3       /* FP64 throughout (checking only: finite-difference gradient checks) */
} dsi_prec;

typedef struct dsi_ctx dsi_ctx; /* device, workspace */
typedef struct dsi_net dsi_net; /* prepared network: packed and cast weights */

#define DSI_MAX_LAYERS 8

/* Architecture of the network (Sec. 4, Sec. 5).  The paper's network is
 * L = 3, C = {1, 64, 32, 1}, k = {11, 11, 11}. */
typedef struct {
  int n1, n2;          /* image rows and columns; N = n1*n2 */
  int M;               /* number of measurements (M >= 1; M < N is typical, not required) */
  int L;               /* number of conv layers, 1..DSI_MAX_LAYERS */
  int C[DSI_MAX_LAYERS + 1]; /* channel counts; C[0] = C[L] = 1 */
  int k[DSI_MAX_LAYERS];     /* odd filter sizes */
  int bias_per_pixel;  /* 1: per-pixel bias [Cout][n1][n2] -- Eq. (1)'s full-grid bias after
                          the crop S, whose border entries never reach the output;
                          0: one bias per output channel [Cout] */
  int relu_last;       /* 1: ReLU after the last layer as well (Sec. 4 applies ReLU in every
                          layer); 0: linear last layer, so signed signals stay representable */
  int fc_trainable;    /* 1: the fully connected layer W_fc is learned too (Sec. 4 notes that
                          it could be); 0: it stays fixed at its given value (Phi^T in the paper) */
} dsi_net_desc;

/* Parameters Omega (Sec. 4), FP32.  Device pointers.  For dsi_net_prepare and
 * dsi_net_update they are read only; for dsi_train_step they are the FP32 master
 * copy, updated in place. */
typedef struct {
  float *w_fc;                  /* [N][M] row-major; Phi^T for the paper's fixed layer */
  float *w[DSI_MAX_LAYERS];     /* [Cout][Cin][k][k] */
  float *b[DSI_MAX_LAYERS];     /* [Cout][n1][n2] if bias_per_pixel, else [Cout] */
} dsi_params;

/* Gradients, same shapes as dsi_params, FP32 device pointers (w_fc written only
 * when the net's fc_trainable is set; it may be NULL otherwise). */
typedef dsi_params dsi_grads;

/* Adam state (Kingma & Ba): first and second moments with the shapes of
 * w[l] and b[l], FP32 device pointers, zero before the first step. */
typedef struct {
  float *m_w[DSI_MAX_LAYERS], *v_w[DSI_MAX_LAYERS];
  float *m_b[DSI_MAX_LAYERS], *v_b[DSI_MAX_LAYERS];
  float beta1, beta2, eps;      /* 0.9, 0.999, 1e-8 */
  long step;                    /* completed steps; dsi_train_step increments it (host field) */
  float *m_fc, *v_fc;           /* [N][M] moments of W_fc (used when fc_trainable) */
} dsi_adam;

/* ------------------------------------------------------------ lifetime */
/* Create a context on HIP device `device`.  *out receives the handle. */
dsi_status dsi_create(dsi_ctx **out, int device);
/* Destroy a context and its workspace.  Waits for the device to go idle. */
dsi_status dsi_destroy(dsi_ctx *ctx);
/* Give the context a caller-owned device workspace of `bytes` bytes (16-byte
 * aligned) instead of the one it allocates and grows itself (which is freed
 * here).  The context never frees or grows caller memory: a later call that
 * needs more than `bytes` (dsi_workspace_size and the training sizes) fails
 * with DSI_E_NOMEM before any launch.  ws = NULL returns to a library-owned
 * workspace, allocated on demand.  The memory must stay valid while the
 * context uses it; calls on the context then use only its first bytes that
 * they need, so a caller may keep other data in its tail (a serving loop
 * keeps its staging buffers there). */
dsi_status dsi_set_workspace(dsi_ctx *ctx, void *ws, size_t bytes);
/* Thread-local message of the last error on this thread ("" if none). */
const char *dsi_last_error(void);
/* Library version string. */
const char *dsi_version(void);

/* ---------------------------------------------------- Sec. 1: y = Phi x */
/* y[b][m] = sum_n phi[m][n] x[b][n], FP32 in and out, FP32 accumulation.
 * phi [M][N], x [B][N], y [B][M].  B = 0 is an empty batch (no-op). */
dsi_status dsi_measure(dsi_ctx *ctx, const float *phi, const float *x, float *y,
                       int B, int M, int N, void *stream);

/* Noisy measurements (Sec. 5, Table 3): y_b = Phi x_b + s_b e_b, with the
 * noise draw e [B][M] (caller-supplied, device) scaled per vector so that
 * ||Phi x_b||^2 / ||s_b e_b||^2 = 10^(snr_db/10).  Other arguments as
 * dsi_measure. */
dsi_status dsi_measure_noisy(dsi_ctx *ctx, const float *phi, const float *x, const float *e,
                             double snr_db, float *y, int B, int M, int N, void *stream);

/* ------------------------------------------- Sec. 4: the recovery network */
/* Validate `desc`, copy and pack `params` into the precision `prec`, and
 * return a prepared network in *out.  The packed copies are owned by the
 * network; `params` may be freed afterwards.  Runs on `stream` and waits for
 * it before returning.  Precisions: DSI_F32 and DSI_F64 for every
 * architecture; DSI_FP8_E4M3 for the paper's architecture (C = {1,64,32,1},
 * k = 11); DSI_BF16 for the paper's architecture and for any other stack of
 * 11 x 11 layers whose hidden widths are 32 or 64 channels (deeper or wider
 * DeepInverse networks, which Sec. 5 leaves to future work: recovery only, their
 * training calls return DSI_E_DTYPE); else DSI_E_DTYPE. */
dsi_status dsi_net_prepare(dsi_ctx *ctx, const dsi_net_desc *desc, const dsi_params *params,
                           dsi_prec prec, dsi_net **out, void *stream);
/* Re-pack the network's copies from new parameter values (same shapes). Enqueued on stream. */
dsi_status dsi_net_update(dsi_ctx *ctx, dsi_net *net, const dsi_params *params, void *stream);
/* FP8 only: static per-tensor activation scales (host array of L+1 floats,
 * the inputs of the proxy layer and of conv layers 1..L: {s_y, s_x~, s_a1,
 * s_a2}), each a positive power of two; a tensor v is stored as the e4m3
 * code of v / s.  The FP8 network quantises y (s_y) and the input of conv
 * layer 2 (s_a1); conv layers 1 and 3 run in BF16, so s_x~ and s_a2 are
 * unused.  Weight scales are set by dsi_net_prepare from the weights'
 * largest magnitude.  Without this call (or dsi_net_calibrate) every
 * activation scale is 1. */
dsi_status dsi_net_set_act_scales(dsi_net *net, const float *scales_host, int n);
/* FP8 only: set the activation scales from a calibration batch y [B][M]:
 * s = 2^ceil(log2(amax / 448)) of y and of conv layer 1's output (computed
 * by the FP8 proxy and the BF16 conv layer 1).  The scales stay fixed
 * afterwards, so a result does not depend on the other images of its batch.
 * Synchronous (waits for `stream`). */
dsi_status dsi_net_calibrate(dsi_ctx *ctx, dsi_net *net, const float *y, int B, void *stream);
/* Scales of a network (host array of n floats): {W_fc, W2, s_y, s_x~, s_a1, s_a2}
 * (weight scales are 1 except for FP8 nets). */
dsi_status dsi_net_get_scales(const dsi_net *net, float *scales, int n);
/* Free a prepared network (device memory is released after the device idles). */
dsi_status dsi_net_free(dsi_ctx *ctx, dsi_net *net);
/* Query the net's precision and description (host outputs, nullable). */
dsi_status dsi_net_info(const dsi_net *net, dsi_net_desc *desc, dsi_prec *prec);

/* Bytes of state one batch of B images needs: train = 1, the saved state of
 * dsi_forward_train that keeps every activation (recompute = 0); train = 2, the
 * saved state of the recompute mode (recompute = 1: the proxy x~, the network's
 * output and, for a trainable FC layer, y -- 2 + 4 bytes per pixel and image in
 * BF16, against 2 + 128 + 64 + 4 with the hidden activations kept); train = 0, the
 * recovery workspace of dsi_recover. */
dsi_status dsi_workspace_size(const dsi_net *net, int B, int train, size_t *bytes);
/* Grow the context's workspace now to serve batches of up to B images of this
 * net (so later calls do not allocate, e.g. under stream capture). Synchronous. */
dsi_status dsi_reserve(dsi_ctx *ctx, const dsi_net *net, int B, int train);

/* xhat = M(y, Omega) (Sec. 4): proxy x~ = W_fc y, then every conv layer of
 * Eq. (1).  y [B][M] FP32, xhat [B][n1][n2] FP32.  B = 0 is a no-op. */
dsi_status dsi_recover(dsi_ctx *ctx, const dsi_net *net, const float *y, float *xhat, int B,
                       void *stream);

/* Size of the fixed device workspace of dsi_recover_noalloc: 64 MiB per device. */
#define DSI_NOALLOC_SCRATCH_BYTES (64L << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): dsi_recover with the
 * same arguments, kernels and results, whose workspace is a fixed device array
 * inside the library (DSI_NOALLOC_SCRATCH_BYTES on each device, held until the
 * process ends; its address is looked up once per device by dsi_create).  It
 * calls no allocating routine.  The workspace a batch needs is
 * dsi_workspace_size(net, B, 0) bytes (about 0.76 MiB per 64 x 64 BF16 image,
 * so B <= 84 at 64 x 64 and B <= 20 at 128 x 128); a larger batch fails with
 * DSI_E_SHAPE before any launch and leaves xhat untouched.  Every call on one
 * device shares that device's array, which keeps the last call's contents:
 * calls that overlap on one GPU (different streams, contexts or threads) race,
 * so order them on one stream.  No stage timing is recorded. */
dsi_status dsi_recover_noalloc(dsi_ctx *ctx, const dsi_net *net, const float *y, float *xhat, int B,
                               void *stream);

/* ------------------------------------------------- Sec. 4: backpropagation */
/* Forward pass that also keeps, in `saved` (caller-owned device buffer of at
 * least dsi_workspace_size(net, B, 1 + recompute) bytes), what the backward pass
 * needs.  recompute = 0: every activation.  recompute = 1: only the proxy x~
 * and the output (and y for a trainable FC layer); the backward pass recomputes
 * the hidden layers from x~ (Sec. 4's backpropagation needs them; recomputing
 * trades their memory for one more pass through conv layers 1..L-1).  In this
 * mode the batch runs in chunks through the context's workspace, as many images
 * per chunk as dsi_set_recompute_budget allows (the whole batch by default), so
 * a batch whose activations outgrow the device still trains.  xhat [B][n1][n2]. */
dsi_status dsi_forward_train(dsi_ctx *ctx, const dsi_net *net, const float *y, float *xhat,
                             int B, void *saved, size_t saved_bytes, int recompute, void *stream);
/* Backward pass of a loss with gradient gxhat = dL/dxhat [B][n1][n2] (FP32),
 * from the state dsi_forward_train left in `saved` for the same y, B and
 * recompute flag.  Writes dL/dw[l] and dL/db[l] into grads (overwriting) and,
 * if gy is not NULL, dL/dy [B][M].  Parameter gradients are summed over the
 * batch in a fixed order, so repeated calls give identical bits.  recompute = 1
 * recomputes the hidden activations chunk by chunk (chunks as in
 * dsi_forward_train); with one chunk the gradients are bit-identical to the
 * recompute = 0 ones, with several the chunks' gradients are added in chunk
 * order (the same sums, reassociated in FP32). */
dsi_status dsi_backward(dsi_ctx *ctx, const dsi_net *net, const float *gxhat, const void *saved,
                        size_t saved_bytes, int recompute, int B, const dsi_grads *grads, float *gy,
                        void *stream);
/* Workspace bytes one chunk of the recompute mode may use on this context: the
 * chunk is the largest number of images whose training state, backward scratch
 * and gradient buffers fit (at least one image).  0 (the default): the whole
 * batch is one chunk. */
dsi_status dsi_set_recompute_budget(dsi_ctx *ctx, size_t bytes);
/* Copy activation `layer` of the state dsi_forward_train (recompute = 0) left in `saved`
 * (0 = the proxy x~, 1..L-1 = the hidden feature maps after ReLU, L = xhat),
 * converted to FP32, into out [B][C_layer][n1][n2] (planar, device). */
dsi_status dsi_saved_activation(dsi_ctx *ctx, const dsi_net *net, const void *saved,
                                size_t saved_bytes, int B, int layer, float *out, void *stream);
/* Loss L = (1/B) sum_b ||xhat_b - x_b||^2 (Sec. 4, accumulated in FP64) and
 * its gradient with respect to every parameter (into grads, overwriting) and,
 * if gy is not NULL, to y [B][M]: forward, dL/dxhat = (2/B)(xhat - x), backward.
 * loss_dev (nullable) is a device double that receives L. */
dsi_status dsi_loss_grad(dsi_ctx *ctx, dsi_net *net, const float *y, const float *x, int B,
                         const dsi_grads *grads, float *gy, double *loss_dev, void *stream);
/* One training step on a batch (Sec. 4): forward in the net's precision, loss
 * L = (1/B) sum_b ||xhat_b - x_b||^2 (accumulated in FP64), backward, Adam
 * update (lr) of the FP32 master parameters `params` (w and b, and w_fc when
 * the net's fc_trainable is set; otherwise w_fc stays fixed, as in the
 * paper's experiments), and a re-pack of the net from them.  y [B][M],
 * x [B][n1][n2].  loss_dev (nullable) is a device double that receives L.
 * opt->step is incremented on the host. */
dsi_status dsi_train_step(dsi_ctx *ctx, dsi_net *net, const dsi_params *params, dsi_adam *opt,
                          const float *y, const float *x, int B, float lr, double *loss_dev,
                          void *stream);

/* ---------------------------------------------------- Sec. 5: metrics */
/* Per image b, in FP64 on the device, out[b][4] =
 *   { ||xhat_b - x_b||^2,
 *     PSNR = 10 log10(max_p x_b[p]^2 / MSE_b)   (Sec. 5 footnote),
 *     ||xhat_b - x_b|| / ||x_b||,
 *     success phi = 1 if ||xhat_b - x_b||^2 / ||x_b||^2 <= 0.1 else 0  (Sec. 5) }.
 * xhat, x [B][N] FP32; out [B][4] device doubles. */
dsi_status dsi_metrics(dsi_ctx *ctx, const float *xhat, const float *x, int B, int N,
                       double *out, void *stream);

/* ---------------------------------------------------- benchmarking */
/* When enabled, every forward pass through the paper's network records HIP
 * events on the caller's stream at the boundaries of its stages {proxy GEMM,
 * conv layer 1, conv layer 2, conv layer 3}: one before the pass's first kernel,
 * one after each stage.  The events are timing-only (no system-scope fence), so
 * recording them does not write the caches back between stages. */
dsi_status dsi_set_stage_timing(dsi_ctx *ctx, int enable);
/* The same for a subset of the stages: bit k of `stages` times stage k (bit 0 the
 * proxy GEMM, bit k >= 1 conv layer k); only the boundaries of timed stages get an
 * event, so fewer stages disturb the pass less.  0 turns timing off. */
dsi_status dsi_set_stage_timing_mask(dsi_ctx *ctx, unsigned stages);
/* Waits for the recorded events, writes the milliseconds spent in each of the
 * first `nstages` stages summed over the timed passes into ms (host array) and
 * their number into *calls (host), then forgets them. */
dsi_status dsi_stage_times(dsi_ctx *ctx, double *ms, int nstages, int *calls);
/* The same per pass: ms (host array of max_passes * (nstages + 1)) receives, in
 * row p = 0 .. min(*calls, max_passes) - 1 of nstages + 1 columns, stage k of the
 * p-th timed pass at ms[p * (nstages + 1) + k] (0 for a stage not timed) and, in
 * the last column, the time from that pass's first event to the next timed pass's
 * first event (0 for the last pass).  Other entries are 0; *calls (host) = the
 * number of timed passes.  Forgets every recorded event, also those of passes
 * beyond max_passes.
 * Errors (these timing calls): DSI_E_NULL for a NULL ctx, ms or calls; DSI_E_SHAPE
 * for nstages < 1 or max_passes < 1; DSI_E_HIP when an event cannot be waited for
 * (the events are forgotten all the same). */
dsi_status dsi_stage_times_each(dsi_ctx *ctx, double *ms, int nstages, int max_passes, int *calls);

#ifdef __cplusplus
}
#endif
#endif /* DSI_H */
