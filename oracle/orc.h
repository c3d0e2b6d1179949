/*
 * orc.h -- FP64 CPU oracle for DeepInverse (Mousavi & Baraniuk, arXiv 1701.03891).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and must never be used as a
 * fallback for it.
 *
 * Everything is plain double precision, written as the definitions in the
 * paper state them, with no blocking or reordering:
 *   - measurement  y = Phi x                                   (Sec. 1)
 *   - signal proxy x~ = Phi^T y, by a fixed fully connected layer (Sec. 4)
 *   - conv layer   S(ReLU(W * x + b)), full 2-D correlation over the
 *                  zero-padded input, bias over the full-size grid, ReLU,
 *                  crop S of the padding borders                 (Sec. 4, Eq. 1)
 *   - loss         L = (1/l) sum_i ||M(y_i) - x_i||^2            (Sec. 4)
 *   - gradients by backpropagation of L                          (Sec. 4)
 *   - Adam update (Kingma & Ba), PSNR (Sec. 5 footnote), success indicator
 *     phi = I(||xhat - x||^2 / ||x||^2 <= 0.1)                    (Sec. 5)
 *   - ISTA in the orthonormal 2-D DCT basis: the sparsity-regularised convex
 *     recovery that Sec. 1 cites, as the classical reference.
 *
 * Layouts: images are row-major n1 x n2 (pixel p = i*n2 + j); feature maps
 * are planar [C][n1][n2] per image; weights are [Cout][Cin][k][k]; "full"
 * biases are [Cout][n1+k-1][n2+k-1] (the size Eq. 1 gives them), channel
 * biases are [Cout].  Batches are the outermost index.
 *
 * Parity unpinned: none of these functions -- every one is pinned by a
 * closed form, an invariant, a library routine or brute force in the
 * test-suite's oracle tests.
 */
#ifndef ORC_H
#define ORC_H

#ifdef __cplusplus
extern "C" {
#endif

/* Network description: L conv layers, channels C[0..L], odd filter sizes k[0..L-1]. */
typedef struct {
  int n1, n2;   /* image rows and columns, N = n1*n2 */
  int M;        /* number of measurements */
  int L;        /* number of conv layers */
  int C[9];     /* channel counts, C[0] = C[L] = 1 */
  int k[8];     /* filter sizes (odd) */
  int bias_full;/* 1: per-pixel bias over the full (n+k-1) grid, 0: per channel */
  int relu_last;/* 1: ReLU on the last layer too */
} orc_net;

/* y[b][m] = sum_n phi[m][n] x[b][n]                                    (Sec. 1) */
void orc_measure(const double *phi, const double *x, double *y, int B, int M, int N);

/* Noisy measurements (Sec. 5, Table 3): y_b += s_b e_b, s_b such that
 * ||y_b||^2 / ||s_b e_b||^2 = 10^(snr_db/10).  e [B][M] is the noise draw. */
void orc_add_noise(double *y, const double *e, int B, int M, double snr_db);

/* xt[b][p] = sum_m wfc[p][m] y[b][m]; wfc = Phi^T, shape [N][M]         (Sec. 4) */
void orc_proxy(const double *wfc, const double *y, double *xt, int B, int M, int N);

/* One conv layer of Eq. (1) on ONE image.  in [Cin][n1][n2], w [Cout][Cin][k][k],
 * bias [Cout][n1+k-1][n2+k-1] (bias_full) or [Cout].  zfull (nullable) receives
 * the full-size pre-activation [Cout][n1+k-1][n2+k-1]; out [Cout][n1][n2]. */
void orc_conv_layer(const double *in, int Cin, int n1, int n2, const double *w, int Cout,
                    int k, const double *bias, int bias_full, int relu, double *zfull,
                    double *out);

/* Bytes of doubles needed per image to keep all activations (for orc_forward's acts). */
long orc_acts_per_image(const orc_net *net);

/* Forward map xhat = M(y, Omega) for a batch.  w[l], b[l] as in orc_conv_layer.
 * acts (nullable): per image, orc_acts_per_image doubles holding a_0..a_L and
 * the full-size pre-activations z_1..z_L, in that order. */
void orc_forward(const orc_net *net, const double *wfc, const double *const *w,
                 const double *const *b, const double *y, int B, double *xhat, double *acts);

/* Reduced-precision operands.  A quantisation point stores a value v as
 * round(v / scale) * scale, round being round-to-nearest-even into the format
 * (ORC_Q_BF16: 8 significand bits, the range of FP32; ORC_Q_E4M3: OCP FP8 e4m3fn,
 * 4 significand bits, subnormals below 2^-6, saturating at +-448). */
enum { ORC_Q_NONE = 0, ORC_Q_BF16 = 1, ORC_Q_E4M3 = 2 };
typedef struct { int fmt; double scale; } orc_q;
typedef struct {
  orc_q y, wfc, xt;   /* measurement vector, fully connected weights, proxy x~ */
  orc_q w[8];         /* conv weights of layer l */
  orc_q a[8];         /* output of conv layer l (after the ReLU) */
  int acc_fp32;       /* error model only: sums are accumulated in FP32 */
} orc_quant;

/* v rounded into format fmt (no scale). */
double orc_round(double v, int fmt);
/* out[i] = round(x[i] / scale) * scale. */
void orc_quantize(const double *x, double *out, long n, int fmt, double scale);
/* The forward map with every operand rounded where qs says, sums exact: y, W_fc and
 * the conv weights are rounded before use, x~ and each layer's output after it is
 * computed.  With every point ORC_Q_NONE it is orc_forward.  sigma (nullable) [B][N]
 * receives a model of the standard deviation of each output pixel's error against
 * the exact forward map: every rounding is an independent error, uniform over one
 * spacing of its format, propagated through the layers to first order; with
 * acc_fp32 the rounding of FP32 running sums is added. */
void orc_forward_q(const orc_net *net, const double *wfc, const double *const *w,
                   const double *const *b, const double *y, int B, const orc_quant *qs,
                   double *xhat, double *sigma);

/* L = (1/B) sum_b ||xhat_b - x_b||^2; g (nullable) = dL/dxhat = (2/B)(xhat - x). */
double orc_loss(const double *xhat, const double *x, int B, int N, double *g);

/* Loss and gradients of L with respect to every parameter, by backpropagation.
 * gw[l], gb[l] have the shapes of w[l], b[l]; gy [B][M] and gwfc [N][M] are
 * nullable.  Returns L. */
double orc_backward(const orc_net *net, const double *wfc, const double *const *w,
                    const double *const *b, const double *y, const double *x, int B,
                    double *const *gw, double *const *gb, double *gy, double *gwfc);

/* Backpropagation from given activations: acts holds, per image, a_0..a_L
 * planar ([C_l][n1][n2] each, concatenated; a_0 the proxy, a_L the output)
 * and g_out = dL/dxhat [B][N].  The ReLU masks are taken from the given
 * post-activations.  Same gradients as orc_backward when the activations are
 * the oracle's own forward ones. */
void orc_backward_acts(const orc_net *net, const double *wfc, const double *const *w,
                       const double *y, const double *acts, const double *g_out, int B,
                       double *const *gw, double *const *gb, double *gy, double *gwfc);

/* One Adam step (Kingma & Ba) on n parameters; t is the 1-based step count. */
void orc_adam(double *theta, const double *g, double *m, double *v, long n, long t,
              double lr, double beta1, double beta2, double eps);

/* PSNR = 10 log10(peak^2 / MSE) with peak = max_p x[p] (Sec. 5 footnote). */
double orc_psnr(const double *xhat, const double *x, int N);
/* ||a - ref||_2 / ||ref||_2 (absolute error when ||ref|| = 0). */
double orc_relerr(const double *a, const double *ref, int N);
/* Success indicator of Sec. 5: 1 if ||xhat - x||^2 / ||x||^2 <= thr. */
int orc_success(const double *xhat, const double *x, int N, double thr);

/* Orthonormal DCT-II matrix C[k][i] = a_k cos(pi (2i+1) k / 2n), a_0 = sqrt(1/n),
 * a_k = sqrt(2/n).  2-D: coefficients S = C X C^T, image X = C^T S C. */
void orc_dct_matrix(int n, double *C);

/* Largest singular value of phi [M][N] by power iteration. */
double orc_spectral_norm(const double *phi, int M, int N, int iters);

/* ISTA (iterative soft thresholding) for min 1/2||y - A s||^2 + lam ||s||_1
 * with A = Phi Psi, Psi the 2-D orthonormal inverse DCT on n1 x n2 images.
 * Continuation: lam_0 = 0.5 ||A^T y||_inf, `stages` stages of `iters`
 * iterations, lam <- decay * lam between stages; then a least-squares debias
 * on the support {|s_j| > 1e-6 max|s|}.  s and x receive the coefficients
 * [n1][n2] and the image [n1][n2].  Returns the support size. */
int orc_ista_dct(const double *phi, const double *y, int M, int n1, int n2, int stages,
                 int iters, double decay, double *s, double *x);
/* orc_ista_dct on B measurement vectors Y [B][M] at once (each image through the
 * same steps and sums as a single run; the passes over Phi are shared).  S, X
 * [B][n1 n2]; supp [B] (nullable) receives the support sizes. */
void orc_ista_dct_batch(const double *phi, const double *Y, int B, int M, int n1, int n2, int stages,
                        int iters, double decay, double *S, double *X, int *supp);

#ifdef __cplusplus
}
#endif
#endif
