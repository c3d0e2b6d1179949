// misc.hip -- weight packing, casts, the loss and its gradient, Sec. 5
// metrics, and the Adam update (Kingma & Ba).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace dsi {

#define GRID1(n) (unsigned)(((long)(n) + 255) / 256), 256

// ------------------------------------------------------------- packing
// W_fc [N][M] fp32 -> [N][Mpad] T, zero-padded columns (K of the proxy GEMM).
template <typename T>
__global__ void pack_fc_kernel(const float *__restrict__ w, T *__restrict__ out, int N, int M, int Mpad) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)N * Mpad) return;
  const int p = (int)(idx / Mpad), m = (int)(idx % Mpad);
  out[idx] = from_f32<T>(m < M ? w[(long)p * M + m] : 0.0f);
}

// conv_mid weights: W [COUT][CIN][11][11] -> [CIN/16][11 v][11 u][COUT/32][64][8].
// flip = 1 packs the data-gradient operator instead: W'[ci][co][u][v] = W[co][ci][10-u][10-v]
// (so COUT/CIN below are those of the operator being packed).
DSI_INLINE float pack_mid_val(const float *__restrict__ w, long idx, int CIN, int COUT, int flip) {
  const int e = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
  long rest = idx >> 9;
  const int nct = COUT / 32;
  const int ct = (int)(rest % nct); rest /= nct;
  const int u = (int)(rest % 11); rest /= 11;
  const int v = (int)(rest % 11); rest /= 11;
  const int cs = (int)rest;
  const int co = ct * 32 + (lane & 31), ci = cs * 16 + (lane >> 5) * 8 + e;
  if (!flip) return w[(((long)co * CIN + ci) * 11 + u) * 11 + v];
  return w[(((long)ci * COUT + co) * 11 + (10 - u)) * 11 + (10 - v)];  // original W[ci][co] (its Cout = CIN here)
}
template <typename T>
__global__ void pack_mid_kernel(const float *__restrict__ w, T *__restrict__ out, int CIN, int COUT, int flip) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)CIN * COUT * 121) return;
  out[idx] = from_f32<T>(pack_mid_val(w, idx, CIN, COUT, flip));
}

// conv_first weights: W [COUT][1][11][11] -> [11 u][COUT/32][64][8], taps v = 8*(lane/32) + e.
// flip = 1 packs the data-gradient operator of a (COUT -> 1) layer instead, whose
// weights [1][COUT][11][11] have the same linear order: W'[c][0][u][v] = W[0][c][10-u][10-v].
DSI_INLINE float pack_first_val(const float *__restrict__ w, int idx, int COUT, int flip) {
  const int nct = COUT / 32;
  const int e = idx & 7, lane = (idx >> 3) & 63, ct = (idx >> 9) % nct, u = (idx >> 9) / nct;
  const int co = ct * 32 + (lane & 31), v = 8 * (lane >> 5) + e;
  if (v >= 11) return 0.0f;
  return flip ? w[((long)co * 11 + (10 - u)) * 11 + (10 - v)] : w[((long)co * 11 + u) * 11 + v];
}
template <typename T>
__global__ void pack_first_kernel(const float *__restrict__ w, T *__restrict__ out, int COUT, int flip) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 11 * (COUT / 32) * 64 * 8) return;
  out[idx] = from_f32<T>(pack_first_val(w, idx, COUT, flip));
}

// conv_last weights: W [1][CIN][11][11] -> [11 v][11 u][CIN].
// flip = 1 packs the data-gradient operator of a (1 -> CIN) layer instead:
// W'[0][c][u][v] = W[c][0][10-u][10-v].
DSI_INLINE float pack_last_val(const float *__restrict__ w, int idx, int CIN, int flip) {
  const int c = idx % CIN, u = (idx / CIN) % 11, v = idx / CIN / 11;
  return flip ? w[((long)c * 11 + (10 - u)) * 11 + (10 - v)] : w[((long)c * 11 + u) * 11 + v];
}
template <typename T>
__global__ void pack_last_kernel(const float *__restrict__ w, T *__restrict__ out, int CIN, int flip) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= CIN * 121) return;
  out[idx] = from_f32<T>(pack_last_val(w, idx, CIN, flip));
}

// Per-pixel bias [C][HW] -> fragment order [HW][C/32][2][4][4]: element idx = pix * C + pos
// comes from channel 32c + 8q + 4h + e, (c, h, q, e) the digits of pos.
DSI_INLINE long bias_frag_src(long idx, int C, long HW) {
  const long pix = idx / C;
  const int pos = (int)(idx % C), r = pos % 32;
  const int ch = 32 * (pos / 32) + 8 * ((r / 4) % 4) + 4 * (r / 16) + r % 4;
  return (long)ch * HW + pix;
}
__global__ void pack_bias_frag_kernel(const float *__restrict__ b, float *__restrict__ out, int C, long HW) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx < (long)C * HW) out[idx] = b[bias_frag_src(idx, C, HW)];
}
hipError_t pack_bias_frag(const float *b, float *out, int C, long HW, hipStream_t s) {
  pack_bias_frag_kernel<<<GRID1((long)C * HW), 0, s>>>(b, out, C, HW);
  return hipGetLastError();
}

// Every packed operand of the paper's network (the three forward layers, the three
// data-gradient operators) and the copies of the three bias tensors, in one launch:
// element ranges follow each other in the order of PaperPack's fields.
template <typename T>
__global__ void pack_paper_kernel(PaperPack pk) {
  long idx = (long)blockIdx.x * 256 + threadIdx.x;
  const long n1 = 11L * 2 * 64 * 8, n2 = 64L * 32 * 121, n3 = 32L * 121, n1f = 11L * 64 * 8, n2f = n2, n3f = 64L * 121;
  if (idx < n1) { ((T *)pk.wp1)[idx] = from_f32<T>(pack_first_val(pk.w[0], (int)idx, 64, 0)); return; }
  idx -= n1;
  if (idx < n2) { ((T *)pk.wp2)[idx] = from_f32<T>(pack_mid_val(pk.w[1], idx, 64, 32, 0)); return; }
  idx -= n2;
  if (idx < n3) { ((T *)pk.wp3)[idx] = from_f32<T>(pack_last_val(pk.w[2], (int)idx, 32, 0)); return; }
  idx -= n3;
  if (idx < n1f) { ((T *)pk.wp3f)[idx] = from_f32<T>(pack_first_val(pk.w[2], (int)idx, 32, 1)); return; }
  idx -= n1f;
  if (idx < n2f) { ((T *)pk.wp2f)[idx] = from_f32<T>(pack_mid_val(pk.w[1], idx, 32, 64, 1)); return; }
  idx -= n2f;
  if (idx < n3f) { ((T *)pk.wp1f)[idx] = from_f32<T>(pack_last_val(pk.w[0], (int)idx, 64, 1)); return; }
  idx -= n3f;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (idx < pk.bn[l]) {
      pk.bp[l][idx] = pk.b[l][l == 1 && pk.hw2 ? bias_frag_src(idx, 32, pk.hw2) : idx];
      return;
    }
    idx -= pk.bn[l];
  }
}
long pack_paper_count(const PaperPack &pk) {
  return 11L * 2 * 64 * 8 + 2 * 64L * 32 * 121 + 32L * 121 + 11L * 64 * 8 + 64L * 121 + pk.bn[0] + pk.bn[1] + pk.bn[2];
}
hipError_t pack_paper(const PaperPack &pk, int prec, hipStream_t s) {
  const long n = pack_paper_count(pk);
  if (prec == 1) pack_paper_kernel<bf16><<<GRID1(n), 0, s>>>(pk);
  else pack_paper_kernel<float><<<GRID1(n), 0, s>>>(pk);
  return hipGetLastError();
}

// per-pixel bias [C][H][W] -> [H][W][C]
__global__ void pack_bias_hwc_kernel(const float *__restrict__ b, float *__restrict__ out, int C, int HW) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)C * HW) return;
  const int c = (int)(idx % C), p = (int)(idx / C);
  out[idx] = b[(long)c * HW + p];
}

template <typename TI, typename TO>
__global__ void cast_kernel(const TI *__restrict__ in, TO *__restrict__ out, long n) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx < n) out[idx] = (TO)in[idx];
}

// y [B][M] fp32 -> [B][Mpad] T (zero-padded), the proxy GEMM's padded operand
template <typename T>
__global__ void pad_rows_kernel(const float *__restrict__ in, T *__restrict__ out, int B, int M, int Mpad) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)B * Mpad) return;
  const int b = (int)(idx / Mpad), m = (int)(idx % Mpad);
  out[idx] = from_f32<T>(m < M ? in[(long)b * M + m] : 0.0f);
}

hipError_t pack_fc(const float *w, void *out, int N, int M, int Mpad, int prec, hipStream_t s) {
  const long n = (long)N * Mpad;
  if (prec == 1) pack_fc_kernel<bf16><<<GRID1(n), 0, s>>>(w, (bf16 *)out, N, M, Mpad);
  else pack_fc_kernel<float><<<GRID1(n), 0, s>>>(w, (float *)out, N, M, Mpad);
  return hipGetLastError();
}
hipError_t pack_mid(const float *w, void *out, int CIN, int COUT, int flip, int prec, hipStream_t s) {
  const long n = (long)CIN * COUT * 121;
  if (prec == 1) pack_mid_kernel<bf16><<<GRID1(n), 0, s>>>(w, (bf16 *)out, CIN, COUT, flip);
  else pack_mid_kernel<float><<<GRID1(n), 0, s>>>(w, (float *)out, CIN, COUT, flip);
  return hipGetLastError();
}
hipError_t pack_first(const float *w, void *out, int COUT, int flip, int prec, hipStream_t s) {
  const int n = 11 * (COUT / 32) * 64 * 8;
  if (prec == 1) pack_first_kernel<bf16><<<GRID1(n), 0, s>>>(w, (bf16 *)out, COUT, flip);
  else pack_first_kernel<float><<<GRID1(n), 0, s>>>(w, (float *)out, COUT, flip);
  return hipGetLastError();
}
hipError_t pack_last(const float *w, void *out, int CIN, int flip, int prec, hipStream_t s) {
  if (prec == 1) pack_last_kernel<bf16><<<GRID1(CIN * 121), 0, s>>>(w, (bf16 *)out, CIN, flip);
  else pack_last_kernel<float><<<GRID1(CIN * 121), 0, s>>>(w, (float *)out, CIN, flip);
  return hipGetLastError();
}
hipError_t pack_bias_hwc(const float *b, float *out, int C, int HW, hipStream_t s) {
  pack_bias_hwc_kernel<<<GRID1((long)C * HW), 0, s>>>(b, out, C, HW);
  return hipGetLastError();
}
hipError_t cast_f32_f64(const float *in, double *out, long n, hipStream_t s) {
  if (n > 0) cast_kernel<float, double><<<GRID1(n), 0, s>>>(in, out, n);
  return hipGetLastError();
}
hipError_t cast_f64_f32(const double *in, float *out, long n, hipStream_t s) {
  if (n > 0) cast_kernel<double, float><<<GRID1(n), 0, s>>>(in, out, n);
  return hipGetLastError();
}
hipError_t pad_rows(const float *in, void *out, int B, int M, int Mpad, int prec, hipStream_t s) {
  const long n = (long)B * Mpad;
  if (n <= 0) return hipSuccess;
  if (prec == 1) pad_rows_kernel<bf16><<<GRID1(n), 0, s>>>(in, (bf16 *)out, B, M, Mpad);
  else pad_rows_kernel<float><<<GRID1(n), 0, s>>>(in, (float *)out, B, M, Mpad);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP8
// max |x| over n floats into *out (as the bit pattern of a non-negative float,
// whose unsigned order is the float order); *out must start at 0.
__global__ void amax_kernel(const float *__restrict__ x, long n, unsigned *__restrict__ out) {
  __shared__ float red[256];
  float m = 0.0f;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) m = fmaxf(m, fabsf(x[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}
template <typename T>
__global__ void amax_any_kernel(const T *__restrict__ x, long n, unsigned *__restrict__ out) {
  __shared__ float red[256];
  float m = 0.0f;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) m = fmaxf(m, fabsf(to_f32(x[i])));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}
__global__ void zero_u32_kernel(unsigned *p) { *p = 0u; }

hipError_t amax_f32(const float *x, long n, unsigned *out, hipStream_t s) {
  zero_u32_kernel<<<1, 1, 0, s>>>(out);
  const long blocks = std::min<long>(1024, (n + 255) / 256);
  if (n > 0) amax_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, n, out);
  return hipGetLastError();
}
hipError_t amax_bf16(const bf16 *x, long n, unsigned *out, hipStream_t s) {
  zero_u32_kernel<<<1, 1, 0, s>>>(out);
  const long blocks = std::min<long>(1024, (n + 255) / 256);
  if (n > 0) amax_any_kernel<bf16><<<(unsigned)blocks, 256, 0, s>>>(x, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------- MFMA fragment order
// Z [R][K] fp32 (row stride ld) -> the order a 32x32 MFMA consumes it in: for row
// tile rt (32 rows), k-step ks (2 FE elements) and lane l, the FE elements
//     Z[32 rt + l%32][2 FE ks + FE (l/32) + e],  e < FE,
// scaled by `scale`, zero beyond R or K.  A wave then reads one fragment as one
// contiguous 64 * FE-element run.  Rp (multiple of 32) and Kp (multiple of 2 FE)
// are the padded extents.  FE = 8: bf16 (RNE); FE = 32: FP8 e4m3 codes.
template <typename TD, int FE, bool TRANS>
__global__ __launch_bounds__(256) void pack_frag_kernel(const float *__restrict__ z, long ld, int R, int K, int Rp,
                                                        int Kp, float scale, TD *__restrict__ out) {
  // A block converts a 32-row x 64-column tile: the loads of a wave read 64 consecutive
  // elements of one row (TRANS: element (r, k) is z[k ld + r], and a wave reads 32
  // consecutive r of two k), the tile passes through LDS (rows padded by 16 bytes against
  // bank conflicts), and each thread then writes whole lane fragments (FE elements, 16 or
  // 32 bytes), 64 lanes of one k-step being one contiguous run.
  constexpr int TC = 64, PAD = 16 / (int)sizeof(TD), NKS = TC / (2 * FE);
  __shared__ __attribute__((aligned(16))) TD t[32][TC + PAD];
  const int tid = threadIdx.x, kb = blockIdx.x * TC, rt = blockIdx.y;
  // every load is issued before any is used (clamped into the matrix; the elements past R
  // or K are replaced by zero afterwards), so they share one round trip
  constexpr int NL = 32 * TC / 256;
  float v[NL];
  auto rc = [&](int e, int &row, int &col) {
    row = TRANS ? e % 32 : e / TC;
    col = TRANS ? e / 32 : e % TC;
  };
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    int row, col;
    rc(j * 256 + tid, row, col);
    const long r = min(rt * 32 + row, R - 1), k = min(kb + col, K - 1);
    v[j] = z[TRANS ? k * ld + r : r * ld + k];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    int row, col;
    rc(j * 256 + tid, row, col);
    const float x = (rt * 32 + row < R && kb + col < K) ? v[j] * scale : 0.0f;
    if constexpr (FE == 8) t[row][col] = from_f32<bf16>(x);
    else t[row][col] = f32_to_e4m3(x);
  }
  __syncthreads();
  const int KS = Kp / (2 * FE), ks0 = kb / (2 * FE);
  for (int f = tid; f < NKS * 64; f += 256) {
    const int g = f / 64, l = f % 64;
    if (ks0 + g >= KS) break;   // (the last tile may reach past Kp, a multiple of 2 FE only)
    const TD *src = &t[l & 31][g * 2 * FE + FE * (l >> 5)];
    TD *dst = out + (((long)rt * KS + ks0 + g) * 64 + l) * FE;
#pragma unroll
    for (int q = 0; q < FE * (int)sizeof(TD) / 16; ++q)
      reinterpret_cast<i32x4 *>(dst)[q] = reinterpret_cast<const i32x4 *>(src)[q];
  }
}
hipError_t pack_frag_bf16(const float *z, long ld, int R, int K, int Rp, int Kp, bf16 *out, hipStream_t s) {
  if (Rp <= 0 || Kp <= 0) return hipSuccess;
  if (R <= 0 || K <= 0) return hipErrorInvalidValue;
  pack_frag_kernel<bf16, 8, false><<<dim3((Kp + 63) / 64, Rp / 32), 256, 0, s>>>(z, ld, R, K, Rp, Kp, 1.0f, out);
  return hipGetLastError();
}
hipError_t pack_frag_bf16_t(const float *z, long ld, int R, int K, int Rp, int Kp, bf16 *out, hipStream_t s) {
  if (Rp <= 0 || Kp <= 0) return hipSuccess;
  if (R <= 0 || K <= 0) return hipErrorInvalidValue;
  pack_frag_kernel<bf16, 8, true><<<dim3((Kp + 63) / 64, Rp / 32), 256, 0, s>>>(z, ld, R, K, Rp, Kp, 1.0f, out);
  return hipGetLastError();
}
hipError_t pack_frag_fp8(const float *z, long ld, int R, int K, int Rp, int Kp, float inv_scale, u8 *out,
                         hipStream_t s) {
  if (Rp <= 0 || Kp <= 0) return hipSuccess;
  if (R <= 0 || K <= 0) return hipErrorInvalidValue;
  pack_frag_kernel<u8, 32, false><<<dim3((Kp + 63) / 64, Rp / 32), 256, 0, s>>>(z, ld, R, K, Rp, Kp, inv_scale, out);
  return hipGetLastError();
}

// W_fc^T [M][N] fp32 from the net's copy of W_fc: fragment-ordered bf16 (frag = 1,
// k-steps of 16 over Mpad) or row-major fp32 [N][Mpad] (frag = 0)
__global__ void fc_transpose_kernel(const void *__restrict__ w, int frag, int N, int M, int Mpad,
                                    float *__restrict__ wT) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)N * M) return;
  const int m = (int)(idx / N), p = (int)(idx % N);
  float v;
  if (frag) {
    const long q = (((long)(p >> 5) * (Mpad / 16) + m / 16) * 64 + (p & 31) + 32 * ((m & 15) >> 3)) * 8 + (m & 7);
    v = (float)reinterpret_cast<const bf16 *>(w)[q];
  } else {
    v = reinterpret_cast<const float *>(w)[(long)p * Mpad + m];
  }
  wT[idx] = v;
}
hipError_t fc_transpose(const void *w, int frag, int N, int M, int Mpad, float *wT, hipStream_t s) {
  const long n = (long)N * M;
  if (n > 0) fc_transpose_kernel<<<GRID1(n), 0, s>>>(w, frag, N, M, Mpad, wT);
  return hipGetLastError();
}

// rows [B][M] fp32 -> FP8 codes [B][Mpad] of in * inv_scale, zero-padded
__global__ void quant_rows_kernel(const float *__restrict__ in, u8 *__restrict__ out, int B, int M, int Mpad,
                                  float inv_scale) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)B * Mpad) return;
  const int b = (int)(idx / Mpad), m = (int)(idx % Mpad);
  out[idx] = m < M ? f32_to_e4m3(in[(long)b * M + m] * inv_scale) : (u8)0;
}
hipError_t quant_rows(const float *in, u8 *out, int B, int M, int Mpad, float inv_scale, hipStream_t s) {
  const long n = (long)B * Mpad;
  if (n > 0) quant_rows_kernel<<<GRID1(n), 0, s>>>(in, out, B, M, Mpad, inv_scale);
  return hipGetLastError();
}

// W2 [32][64][11][11] fp32 -> FP8 codes [11 v][11 u][64 lanes][32]: lane l holds
// W[co = l%32][ci = 32*(l/32) + e][u][v] * inv_scale (one 64-channel slice, one tile of 32 outputs)
__global__ void pack_mid_fp8_kernel(const float *__restrict__ w, u8 *__restrict__ out, float inv_scale) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 32 * 64 * 121) return;
  const int e = idx & 31, lane = (idx >> 5) & 63, u = (idx >> 11) % 11, v = (idx >> 11) / 11;
  const int co = lane & 31, ci = 32 * (lane >> 5) + e;
  out[idx] = f32_to_e4m3(w[(((long)co * 64 + ci) * 11 + u) * 11 + v] * inv_scale);
}
hipError_t pack_mid_fp8(const float *w, u8 *out, float inv_scale, hipStream_t s) {
  pack_mid_fp8_kernel<<<GRID1(32 * 64 * 121), 0, s>>>(w, out, inv_scale);
  return hipGetLastError();
}

// W_fc [N][M] fp32 -> FP8 codes [N][Mpad] (zero-padded)
__global__ void pack_fc_fp8_kernel(const float *__restrict__ w, u8 *__restrict__ out, int N, int M, int Mpad,
                                   float inv_scale) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)N * Mpad) return;
  const int p = (int)(idx / Mpad), m = (int)(idx % Mpad);
  out[idx] = m < M ? f32_to_e4m3(w[(long)p * M + m] * inv_scale) : (u8)0;
}
hipError_t pack_fc_fp8(const float *w, u8 *out, int N, int M, int Mpad, float inv_scale, hipStream_t s) {
  const long n = (long)N * Mpad;
  pack_fc_fp8_kernel<<<GRID1(n), 0, s>>>(w, out, N, M, Mpad, inv_scale);
  return hipGetLastError();
}

// ------------------------------------------------ learnable FC layer gradient
// dW_fc[p][m] = sum_b g[b][p] y[b][m]  (g = dL/dx~ [B][N], y [B][ldy]); fixed order over b.
template <typename TG, typename Acc>
__global__ void fc_wgrad_kernel(const TG *__restrict__ g, const float *__restrict__ y, long ldy, int B, int N, int M,
                                float *__restrict__ dw) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)N * M) return;
  const int p = (int)(idx / M), m = (int)(idx % M);
  Acc s = 0;
  for (int b = 0; b < B; ++b) s += (Acc)g[(long)b * N + p] * (Acc)y[(long)b * ldy + m];
  dw[idx] = (float)s;
}
// out[c][r] = in[r][c] for an R x Cc block of in (row stride ldin); out has row stride R.
// 32 x 32 tiles through LDS (one padding column: conflict-free column reads).
__global__ __launch_bounds__(256) void transpose_f32_kernel(const float *__restrict__ in, long ldin, int R, int Cc,
                                                            float *__restrict__ out) {
  __shared__ float t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    t[ty + 8 * k][tx] = (r < R && c < Cc) ? in[(long)r * ldin + c] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = c0 + ty + 8 * k, r = r0 + tx;
    if (c < Cc && r < R) out[(long)c * R + r] = t[tx][ty + 8 * k];
  }
}

// dW_fc[p][m] = sum_b g[b][p] y[b][m] as the MFMA GEMM C[p][m] = sum_b gT[p][b] yT[m][b]
// (FP32 operands, FP32 accumulation) after transposing g and y into `tmp`
// (N * B + M * B floats).
hipError_t fc_wgrad_f32(const float *g, const float *y, long ldy, int B, int N, int M, float *dw, float *tmp,
                        hipStream_t s) {
  if ((long)N * M <= 0 || B <= 0) return hipSuccess;
  float *gT = tmp, *yT = tmp + (((long)N * B + 63) / 64) * 64;
  transpose_f32_kernel<<<dim3((N + 31) / 32, (B + 31) / 32), 256, 0, s>>>(g, N, B, N, gT);
  transpose_f32_kernel<<<dim3((M + 31) / 32, (B + 31) / 32), 256, 0, s>>>(y, ldy, B, M, yT);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return gemm_nt_f32(gT, B, yT, B, dw, M, N, M, B, B % 16 == 0, s);
}
// BF16 networks: dW_fc = g^T y on the BF16 matrix cores, FP32 accumulation and output.  g^T
// and y^T are packed straight into fragment order (rows p and m, k = the batch), then the
// fragment GEMM runs with N as its rows and M as its columns.
size_t fc_wgrad_bf16_scratch(int B, int N, int M) {
  const size_t kp = ((size_t)B + 15) / 16 * 16;
  return (((size_t)N + 31) / 32 * 32 * kp * 2 + 255) / 256 * 256 + ((size_t)M + 31) / 32 * 32 * kp * 2;
}
hipError_t fc_wgrad_bf16(const float *g, const float *y, long ldy, int B, int N, int M, float *dw, void *tmp,
                         hipStream_t s) {
  if ((long)N * M <= 0 || B <= 0) return hipSuccess;
  const int Kp = (B + 15) / 16 * 16, Np = (N + 31) / 32 * 32, Mp = (M + 31) / 32 * 32;
  bf16 *gp = static_cast<bf16 *>(tmp);
  bf16 *yp = reinterpret_cast<bf16 *>(static_cast<char *>(tmp) + ((size_t)Np * Kp * 2 + 255) / 256 * 256);
  hipError_t e = pack_frag_bf16_t(g, N, N, B, Np, Kp, gp, s);
  if (e == hipSuccess) e = pack_frag_bf16_t(y, ldy, M, B, Mp, Kp, yp, s);
  if (e == hipSuccess) e = gemm_frag_bf16_f32(gp, yp, dw, M, N, M, Kp / 16, s);
  return e;
}
hipError_t fc_wgrad_f64(const double *g, const float *y, long ldy, int B, int N, int M, float *dw, hipStream_t s) {
  const long n = (long)N * M;
  if (n > 0) fc_wgrad_kernel<double, double><<<GRID1(n), 0, s>>>(g, y, ldy, B, N, M, dw);
  return hipGetLastError();
}

// ------------------------------------------------------ noisy measurements
// y_b += s_b e_b with ||y_b||^2 / ||s_b e_b||^2 = 10^(snr_db/10); one block per
// measurement vector, FP64 norms in a fixed order.
__global__ __launch_bounds__(256) void add_noise_kernel(float *__restrict__ y, const float *__restrict__ e, int M,
                                                        double snr_db) {
  __shared__ double ry[256], re[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  double sy = 0.0, se = 0.0;
  for (int m = tid; m < M; m += 256) {
    const double a = y[(long)b * M + m], c = e[(long)b * M + m];
    sy += a * a;
    se += c * c;
  }
  ry[tid] = sy;
  re[tid] = se;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      ry[tid] += ry[tid + h];
      re[tid] += re[tid + h];
    }
    __syncthreads();
  }
  const double s = re[0] > 0.0 ? sqrt(ry[0] / re[0]) * pow(10.0, -snr_db / 20.0) : 0.0;
  for (int m = tid; m < M; m += 256) y[(long)b * M + m] = (float)((double)y[(long)b * M + m] + s * e[(long)b * M + m]);
}
hipError_t add_noise(float *y, const float *e, int B, int M, double snr_db, hipStream_t s) {
  if (B > 0) add_noise_kernel<<<B, 256, 0, s>>>(y, e, M, snr_db);
  return hipGetLastError();
}

// ------------------------------------------------------ loss and metrics
// One block per image, FP64 reductions in a fixed order.
// stats[b][4] = { ||xh-x||^2, PSNR (peak = max x), ||xh-x||/||x||, success (ratio <= 0.1) }
// g (nullable) = scale * (xh - x), masked by (xh > 0) when relu_last.
template <typename TX>
__global__ __launch_bounds__(256) void image_stats_kernel(const TX *__restrict__ xh, const float *__restrict__ x,
                                                          int N, double *__restrict__ stats,
                                                          float *__restrict__ g, double *__restrict__ g64,
                                                          double scale, int relu_last) {
  __shared__ double s_sse[256], s_nx[256], s_mx[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  double sse = 0.0, nx = 0.0, mx = -1e308;
  for (int p = tid; p < N; p += 256) {
    const double a = (double)xh[(long)b * N + p], t = (double)x[(long)b * N + p];
    const double d = a - t;
    sse += d * d;
    nx += t * t;
    mx = t > mx ? t : mx;
    double gv = scale * d;
    if (relu_last && !(a > 0.0)) gv = 0.0;
    if (g) g[(long)b * N + p] = (float)gv;
    if (g64) g64[(long)b * N + p] = gv;
  }
  s_sse[tid] = sse; s_nx[tid] = nx; s_mx[tid] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      s_sse[tid] += s_sse[tid + h];
      s_nx[tid] += s_nx[tid + h];
      s_mx[tid] = s_mx[tid] > s_mx[tid + h] ? s_mx[tid] : s_mx[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0 && stats) {
    const double e = s_sse[0], n2 = s_nx[0], peak = s_mx[0];
    stats[b * 4 + 0] = e;
    stats[b * 4 + 1] = 10.0 * log10(peak * peak / (e / N));
    stats[b * 4 + 2] = n2 > 0.0 ? sqrt(e / n2) : sqrt(e);
    stats[b * 4 + 3] = (e / n2 <= 0.1) ? 1.0 : 0.0;
  }
}

// L = (1/B) sum_b sse_b, summed in image order
// loss = (1/B) sum_b stats[b][0]: thread t sums images t, t+256, ... in order, then a
// fixed pairwise tree over the 256 partial sums (the same result on every run)
__global__ __launch_bounds__(256) void loss_sum_kernel(const double *__restrict__ stats, int B, double *__restrict__ loss) {
  __shared__ double part[256];
  const int t = threadIdx.x;
  double sum = 0.0;
  for (int b = t; b < B; b += 256) sum += stats[(long)b * 4];
  part[t] = sum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) *loss = part[0] / B;
}

hipError_t image_stats_f32(const float *xh, const float *x, int B, int N, double *stats, float *g,
                           double scale, int relu_last, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  image_stats_kernel<float><<<B, 256, 0, s>>>(xh, x, N, stats, g, nullptr, scale, relu_last);
  return hipGetLastError();
}
hipError_t image_stats_f64(const double *xh, const float *x, int B, int N, double *stats, double *g64,
                           double scale, int relu_last, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  image_stats_kernel<double><<<B, 256, 0, s>>>(xh, x, N, stats, nullptr, g64, scale, relu_last);
  return hipGetLastError();
}
hipError_t loss_sum(const double *stats, int B, double *loss, hipStream_t s) {
  loss_sum_kernel<<<1, 256, 0, s>>>(stats, B, loss);
  return hipGetLastError();
}

// g_out = g * (a > 0): gradient through the last layer's ReLU (relu_last)
template <typename TA, typename TO>
__global__ void relu_mask_kernel(const float *__restrict__ g, const TA *__restrict__ a, TO *__restrict__ out, long n) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx < n) out[idx] = (a == nullptr || a[idx] > (TA)0) ? (TO)g[idx] : (TO)0;
}
hipError_t relu_mask_f32(const float *g, const float *a, float *out, long n, hipStream_t s) {
  if (n > 0) relu_mask_kernel<float, float><<<GRID1(n), 0, s>>>(g, a, out, n);
  return hipGetLastError();
}
hipError_t relu_mask_f64(const float *g, const double *a, double *out, long n, hipStream_t s) {
  if (n > 0) relu_mask_kernel<double, double><<<GRID1(n), 0, s>>>(g, a, out, n);
  return hipGetLastError();
}

// dst += src (the gradients of a later chunk of a batch added to the earlier chunks')
__global__ void add_f32_kernel(float *__restrict__ dst, const float *__restrict__ src, long n) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx < n) dst[idx] += src[idx];
}
hipError_t add_f32(float *dst, const float *src, long n, hipStream_t s) {
  if (n > 0) add_f32_kernel<<<GRID1(n), 0, s>>>(dst, src, n);
  return hipGetLastError();
}

// saved activation -> planar fp32 [B][C][H][W]
template <typename TI>
__global__ void unpack_act_kernel(const TI *__restrict__ in, ActView vi, float *__restrict__ out, int B) {
  const long n = (long)B * vi.C * vi.H * vi.W;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int j = (int)(idx % vi.W), i = (int)(idx / vi.W % vi.H), c = (int)(idx / ((long)vi.W * vi.H) % vi.C);
  const int b = (int)(idx / ((long)vi.W * vi.H * vi.C));
  out[idx] = to_f32(in[act_idx(vi, b, c, i, j)]);
}
template <typename TI>
hipError_t unpack_act(const TI *in, ActView vi, float *out, int B, hipStream_t s) {
  const long n = (long)B * vi.C * vi.H * vi.W;
  if (n > 0) unpack_act_kernel<TI><<<GRID1(n), 0, s>>>(in, vi, out, B);
  return hipGetLastError();
}
template hipError_t unpack_act<float>(const float *, ActView, float *, int, hipStream_t);
template hipError_t unpack_act<double>(const double *, ActView, float *, int, hipStream_t);
template hipError_t unpack_act<bf16>(const bf16 *, ActView, float *, int, hipStream_t);

// ------------------------------------------------------------------ Adam
// theta -= lr * mhat / (sqrt(vhat) + eps), mhat = m / c1, vhat = v / c2
DSI_INLINE float adam_one(float &th, float gi, float &m, float &v, float lr, float b1, float b2, float eps, float c1,
                          float c2) {
  const float mi = b1 * m + (1.0f - b1) * gi;
  const float vi = b2 * v + (1.0f - b2) * gi * gi;
  m = mi;
  v = vi;
  th -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  return th;
}
template <typename TG>
__global__ void adam_kernel(float *__restrict__ th, const TG *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  adam_one(th[idx], (float)g[idx], m[idx], v[idx], lr, b1, b2, eps, c1, c2);
}
hipError_t adam_f32(float *th, const float *g, float *m, float *v, long n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s) {
  if (n > 0) adam_kernel<float><<<GRID1(n), 0, s>>>(th, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
// Several tensors in one launch: tensor k owns the flat range [start[k], start[k+1]); its
// updated values are also written to mirror (when given), the network's own copy.
// A thread updates four consecutive elements of one segment (each segment's thread count is
// rounded up, so a group never spans two): 16-byte loads and stores when the group is whole and
// the segment's arrays are 16-byte aligned, element by element otherwise.  Every element takes
// the same arithmetic either way.
__global__ __launch_bounds__(256) void adam_multi_kernel(AdamMulti a, float lr, float b1, float b2, float eps,
                                                         float c1, float c2) {
  long q = (long)blockIdx.x * 256 + threadIdx.x;
  int k = 0;
  while (k < a.nseg && q >= (a.seg[k].n + 3) / 4) {
    q -= (a.seg[k].n + 3) / 4;
    ++k;
  }
  if (k >= a.nseg) return;
  const AdamSeg &sg = a.seg[k];
  const long i0 = 4 * q;
  const unsigned long al = reinterpret_cast<unsigned long>(sg.th) | reinterpret_cast<unsigned long>(sg.g) |
                           reinterpret_cast<unsigned long>(sg.m) | reinterpret_cast<unsigned long>(sg.v) |
                           reinterpret_cast<unsigned long>(sg.mirror);
  if (i0 + 3 < sg.n && (al & 15) == 0) {
    f32x4 th = *reinterpret_cast<const f32x4 *>(sg.th + i0), m = *reinterpret_cast<const f32x4 *>(sg.m + i0);
    f32x4 v = *reinterpret_cast<const f32x4 *>(sg.v + i0);
    const f32x4 g = *reinterpret_cast<const f32x4 *>(sg.g + i0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float te = th[e], me = m[e], ve = v[e];
      adam_one(te, g[e], me, ve, lr, b1, b2, eps, c1, c2);
      th[e] = te;
      m[e] = me;
      v[e] = ve;
    }
    *reinterpret_cast<f32x4 *>(sg.th + i0) = th;
    *reinterpret_cast<f32x4 *>(sg.m + i0) = m;
    *reinterpret_cast<f32x4 *>(sg.v + i0) = v;
    if (sg.mirror) *reinterpret_cast<f32x4 *>(sg.mirror + i0) = th;
  } else {
    for (long i = i0; i < i0 + 4 && i < sg.n; ++i) {
      const float t = adam_one(sg.th[i], sg.g[i], sg.m[i], sg.v[i], lr, b1, b2, eps, c1, c2);
      if (sg.mirror) sg.mirror[i] = t;
    }
  }
}
hipError_t adam_multi(const AdamMulti &a, float lr, float b1, float b2, float eps, float c1, float c2,
                      hipStream_t s) {
  long n = 0;
  for (int k = 0; k < a.nseg; ++k) n += (a.seg[k].n + 3) / 4;
  if (n > 0) adam_multi_kernel<<<GRID1(n), 0, s>>>(a, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace dsi
