// internal.h -- launchers shared between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace dsi {

// Activation tensor view: planar [B][C][H][W] or channel-blocked [B][C/16][H][W][16].
struct ActView {
  int C, H, W;
  int blocked;
};

enum { EPI_BIAS = 0, EPI_MASK = 1 };

__host__ __device__ inline long act_idx(const ActView &v, int b, int c, int i, int j) {
  return v.blocked ? ((((long)b * (v.C >> 4) + (c >> 4)) * v.H + i) * v.W + j) * 16 + (c & 15)
                   : (((long)b * v.C + c) * v.H + i) * v.W + j;
}

// gemm.hip: C[b][o] = sum_k X[b][k] W[o][k]
hipError_t gemm_nt_f32(const float *X, long ldx, const float *W, long ldw, float *C, long ldc,
                       int Bn, int O, int K, bool vec, hipStream_t s);
hipError_t gemm_nt_bf16_out_bf16(const float *X, long ldx, const __bf16 *W, long ldw, __bf16 *C,
                                 long ldc, int Bn, int O, int K, bool vec, hipStream_t s);
hipError_t gemm_nt_bf16_out_f32(const float *X, long ldx, const __bf16 *W, long ldw, float *C,
                                long ldc, int Bn, int O, int K, bool vec, hipStream_t s);
hipError_t gemm_nt_f64(const double *X, long ldx, const double *W, long ldw, double *C, long ldc,
                       int Bn, int O, int K, hipStream_t s);

// conv_direct.hip (any shape)
template <typename TI, typename TW, typename TO, typename Acc>
hipError_t conv_fwd_direct(const TI *in, ActView vi, const TW *w, const TW *bias, int bias_pp,
                           int relu, TO *out, ActView vo, int B, int k, hipStream_t s);
template <typename TG, typename TW, typename TA, typename TO, typename Acc>
hipError_t conv_dgrad_direct(const TG *gz, ActView vg, const TW *w, const TA *amask, ActView va,
                             TO *gin, ActView vo, int B, int k, hipStream_t s);
template <typename TG, typename TI, typename Acc, typename TD>
hipError_t conv_wgrad_direct(const TG *gz, ActView vg, const TI *in, ActView vi, int B, int k,
                             TD *dw, hipStream_t s);
template <typename TG, typename Acc, typename TD>
hipError_t bias_grad(const TG *gz, ActView vg, int B, int per_pixel, TD *db, hipStream_t s);

// conv_mfma.hip (the paper's 1 -> 64 -> 32 -> 1, 11 x 11 network)
template <typename T, int COUT, int EPI, typename TI, typename TO>
hipError_t conv_first(const TI *in, const T *wp, const float *bias, int bias_pp, int relu, const T *mask,
                      TO *out, int B, int H, int W, hipStream_t s, float oscale = 1.0f);
template <typename T, int CIN, int COUT, int EPI, typename TO>
hipError_t conv_mid(const T *in, const T *wp, const float *bias, int bias_pp, int relu, const T *mask,
                    TO *out, int B, int H, int W, hipStream_t s, float oscale = 1.0f);
template <typename T, int CIN>
hipError_t conv_last(const T *in, const T *w, const float *bias, int bias_pp, int relu, float *out, int B,
                     int H, int W, hipStream_t s);

}  // namespace dsi

namespace dsi {
// misc.hip; prec: 0 = fp32, 1 = bf16
hipError_t pack_fc(const float *w, void *out, int N, int M, int Mpad, int prec, hipStream_t s);
hipError_t pack_mid(const float *w, void *out, int CIN, int COUT, int flip, int prec, hipStream_t s);
hipError_t pack_first(const float *w, void *out, int COUT, int flip, int prec, hipStream_t s);
hipError_t pack_last(const float *w, void *out, int CIN, int flip, int prec, hipStream_t s);
// all packed operands of the paper's network and its bias copies, one launch
struct PaperPack {
  const float *w[3];      // OIHW fp32 weights of the three layers
  const float *b[3];      // fp32 biases (caller layout)
  long bn[3];             // bias element counts
  void *wp1, *wp2, *wp3;  // forward operands (T)
  void *wp3f, *wp2f, *wp1f;  // data-gradient operators (T)
  float *bp[3];           // the network's bias copies
  long hw2;               // H * W: layer 2's per-pixel bias goes to fragment order; 0: plain copy
};
// per-pixel bias [C][HW] -> [HW][C/32][2][4][4] (the conv_mid epilogue's order)
hipError_t pack_bias_frag(const float *b, float *out, int C, long HW, hipStream_t s);
hipError_t pack_paper(const PaperPack &pk, int prec, hipStream_t s);
hipError_t pack_bias_hwc(const float *b, float *out, int C, int HW, hipStream_t s);
hipError_t cast_f32_f64(const float *in, double *out, long n, hipStream_t s);
hipError_t cast_f64_f32(const double *in, float *out, long n, hipStream_t s);
hipError_t pad_rows(const float *in, void *out, int B, int M, int Mpad, int prec, hipStream_t s);
hipError_t image_stats_f32(const float *xh, const float *x, int B, int N, double *stats, float *g,
                           double scale, int relu_last, hipStream_t s);
hipError_t image_stats_f64(const double *xh, const float *x, int B, int N, double *stats, double *g64,
                           double scale, int relu_last, hipStream_t s);
hipError_t loss_sum(const double *stats, int B, double *loss, hipStream_t s);
template <typename TI>
hipError_t unpack_act(const TI *in, ActView vi, float *out, int B, hipStream_t s);
// tmp: N * B + M * B floats (+ 64 of alignment) of scratch for the transposed operands
hipError_t fc_wgrad_f32(const float *g, const float *y, long ldy, int B, int N, int M, float *dw, float *tmp,
                        hipStream_t s);
hipError_t fc_wgrad_f64(const double *g, const float *y, long ldy, int B, int N, int M, float *dw, hipStream_t s);
// BF16 networks: dW_fc = g^T y on the BF16 matrix cores (FP32 accumulation and output); tmp holds
// fc_wgrad_bf16_scratch(B, N, M) bytes (256-byte aligned)
size_t fc_wgrad_bf16_scratch(int B, int N, int M);
hipError_t fc_wgrad_bf16(const float *g, const float *y, long ldy, int B, int N, int M, float *dw, void *tmp,
                         hipStream_t s);
hipError_t add_noise(float *y, const float *e, int B, int M, double snr_db, hipStream_t s);
hipError_t relu_mask_f32(const float *g, const float *a, float *out, long n, hipStream_t s);
hipError_t relu_mask_f64(const float *g, const double *a, double *out, long n, hipStream_t s);
hipError_t add_f32(float *dst, const float *src, long n, hipStream_t s);
hipError_t adam_f32(float *th, const float *g, float *m, float *v, long n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s);
struct AdamSeg {
  float *th;
  const float *g;
  float *m, *v;
  long n;
  float *mirror;  // optional second copy of the updated values (nullptr: none)
};
struct AdamMulti {
  AdamSeg seg[2 * 8 + 1];
  int nseg;
};
hipError_t adam_multi(const AdamMulti &a, float lr, float b1, float b2, float eps, float c1, float c2,
                      hipStream_t s);
}  // namespace dsi

namespace dsi {
// conv_bwd.hip: MFMA weight gradients (bf16 operands, fp32 partials reduced in a fixed order)
enum { THIN_OUT = 0, THIN_IN = 1 };
size_t conv_wgrad_mid_partial_floats(int CIN, int nchunk);
hipError_t conv_wgrad_mid(const __bf16 *g, const __bf16 *a, int CIN, float *partial, int nchunk, float *dw, int B,
                          int H, int W, hipStream_t s, bool planar = false);
// x [B][C/16][HW][16] -> [B][C][HW] (bf16), for the channel-major conv2 weight gradient
hipError_t to_planar(const __bf16 *in, __bf16 *out, int B, int C, int HW, hipStream_t s);
size_t conv_wgrad_thin_partial_floats(int CW, int nchunk);
template <typename TT>
hipError_t conv_wgrad_thin(int mode, const __bf16 *wide, const TT *thin, int CW, float *partial, int nchunk, float *dw,
                           int B, int H, int W, hipStream_t s);
}  // namespace dsi

namespace dsi {
// FP8 e4m3 path (gemm.hip, misc.hip)
hipError_t gemm_nt_fp8(const unsigned char *X, long ldx, const unsigned char *W, long ldw, __bf16 *C, long ldc,
                       int Bn, int O, int K, float oscale, hipStream_t s);
hipError_t amax_f32(const float *x, long n, unsigned *out, hipStream_t s);
hipError_t amax_bf16(const __bf16 *x, long n, unsigned *out, hipStream_t s);
hipError_t quant_rows(const float *in, unsigned char *out, int B, int M, int Mpad, float inv_scale, hipStream_t s);
hipError_t pack_frag_bf16(const float *z, long ld, int R, int K, int Rp, int Kp, __bf16 *out, hipStream_t s);
// the same for a transposed source: element (r, k) at z[k ld + r]
hipError_t pack_frag_bf16_t(const float *z, long ld, int R, int K, int Rp, int Kp, __bf16 *out, hipStream_t s);
hipError_t pack_frag_fp8(const float *z, long ld, int R, int K, int Rp, int Kp, float inv_scale, unsigned char *out,
                         hipStream_t s);
hipError_t fc_transpose(const void *w, int frag, int N, int M, int Mpad, float *wT, hipStream_t s);
// C[b][o] = scale * sum_k X[b][k] W[o][k], both operands in MFMA fragment order (pack_frag_*),
// KS k-steps; C [Bn][ldc] bf16
hipError_t gemm_frag_bf16(const __bf16 *Xp, const __bf16 *Wp, __bf16 *C, long ldc, int Bn, int O, int KS, hipStream_t s);
// the same GEMM with an FP32 output (the trainable FC's weight gradient)
hipError_t gemm_frag_bf16_f32(const __bf16 *Xp, const __bf16 *Wp, float *C, long ldc, int Bn, int O, int KS,
                              hipStream_t s);
hipError_t gemm_frag_fp8(const unsigned char *Xp, const unsigned char *Wp, __bf16 *C, long ldc, int Bn, int O, int KS,
                         float scale, hipStream_t s);
hipError_t pack_mid_fp8(const float *w, unsigned char *out, float inv_scale, hipStream_t s);
hipError_t pack_fc_fp8(const float *w, unsigned char *out, int N, int M, int Mpad, float inv_scale, hipStream_t s);
}  // namespace dsi

namespace dsi {
// noalloc.hip: device address of the library's fixed workspace array on `device`
// (which must be the current device), looked up once per device and cached
hipError_t noalloc_scratch(int device, void **ptr);
}  // namespace dsi
