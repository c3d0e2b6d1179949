// conv_bwd.hip -- weight gradient of the paper's 11 x 11 layers with 32 output
// channels on CDNA4 matrix cores (backpropagation of Sec. 4's loss).
//
//   dW[co][ci][u][v] = sum_{b,i,j} g[b][co][i][j] * a[b][ci][i+u-5][j+v-5]
//
// For one tap column v this is, per output row pair (i, i+u-5), a GEMM with
// K = 16 consecutive columns:  D_u[co][ci] += sum_j G[co][i][j] A[ci][i+u-5][j+v-5].
// A block owns (32-channel tile of ci, tap column v, a chunk of images); its
// four waves own four 16-column chunks.  Per strip of 8 output rows the block
// stages G (8 rows) and A (18 rows) in LDS as planar [channel][row][col]
// tiles; a wave keeps the 8 G fragments of the strip in registers and walks
// the 18 A rows once, each A fragment (8 consecutive columns shifted by v - 5,
// an unaligned 16-byte LDS read) feeding up to 8 MFMAs (one per u).
// Accumulators (11 u x 32 x 32) live across all strips and images of the
// block; each block then writes its raw accumulators, and a second kernel sums
// the partials in a fixed order (deterministic).
#include "common.h"
#include "internal.h"

namespace dsi {

constexpr int WG_SR = 8;            // output rows per strip
constexpr int WG_LR = WG_SR + 10;   // input rows per strip
constexpr int WG_TW = 64;           // output columns per pass (4 waves x 16)
constexpr int WG_GW = WG_TW + 8;    // G tile row pitch (elements)
constexpr int WG_AW = WG_TW + 16;   // A tile row pitch: cols -5 .. 74 (+ padding)

// g [B][2][H][W][16] (T), a [B][CIN/16][H][W][16] (T)
// partial [(ct*11 + v)*nchunk + chunk][4 waves][11 u][64 lanes][16] fp32
template <int CIN>
__global__ __launch_bounds__(256) void conv_wgrad_mid_kernel(const bf16 *__restrict__ g, const bf16 *__restrict__ a,
                                                             float *__restrict__ partial, int B, int H, int W,
                                                             int nchunk) {
  __shared__ __attribute__((aligned(16))) bf16 gl[32 * WG_SR * WG_GW];
  __shared__ __attribute__((aligned(16))) bf16 al[32 * WG_LR * WG_AW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c32 = lane & 31;
  const int chunk = blockIdx.x % nchunk, v = (blockIdx.x / nchunk) % 11, ct = blockIdx.x / nchunk / 11;
  const int per = (B + nchunk - 1) / nchunk;
  const int b0 = chunk * per, b1 = min(B, b0 + per);

  f32x16 acc[11];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;

  for (int b = b0; b < b1; ++b)
    for (int i0 = 0; i0 < H; i0 += WG_SR)
      for (int j0 = 0; j0 < W; j0 += WG_TW) {
        __syncthreads();
        // G strip: rows i0..i0+7, cols j0..j0+63, 32 channels (two 16-channel slices)
        for (int idx = tid; idx < WG_SR * WG_TW * 4; idx += 256) {
          const int q = idx & 3, pix = idx >> 2;               // q: 8-channel group
          const int row = pix / WG_TW, col = pix - row * WG_TW;
          const int gi = i0 + row, gj = j0 + col;
          bf16x8 val;
          if (gi < H && gj < W)
            val = *reinterpret_cast<const bf16x8 *>(g + ((((long)b * 2 + (q >> 1)) * H + gi) * W + gj) * 16 + (q & 1) * 8);
          else
            for (int e = 0; e < 8; ++e) val[e] = (bf16)0.0f;
#pragma unroll
          for (int e = 0; e < 8; ++e) gl[((q * 8 + e) * WG_SR + row) * WG_GW + col] = val[e];
        }
        // A strip: rows i0-5..i0+12, cols j0-5..j0+68, channels ct*32..ct*32+31
        for (int idx = tid; idx < WG_LR * (WG_TW + 10) * 4; idx += 256) {
          const int q = idx & 3, pix = idx >> 2;
          const int row = pix / (WG_TW + 10), col = pix - row * (WG_TW + 10);
          const int gi = i0 - 5 + row, gj = j0 - 5 + col;
          const int c0 = ct * 32 + q * 8;
          bf16x8 val;
          if (gi >= 0 && gi < H && gj >= 0 && gj < W)
            val = *reinterpret_cast<const bf16x8 *>(a + ((((long)b * (CIN / 16) + (c0 >> 4)) * H + gi) * W + gj) * 16 + (c0 & 15));
          else
            for (int e = 0; e < 8; ++e) val[e] = (bf16)0.0f;
#pragma unroll
          for (int e = 0; e < 8; ++e) al[((q * 8 + e) * WG_LR + row) * WG_AW + col] = val[e];
        }
        __syncthreads();
        // G fragments of the strip: lane (co = c32, h) holds G[co][i][16w + 8h + e]
        Frag8<bf16> gf[WG_SR];
#pragma unroll
        for (int i = 0; i < WG_SR; ++i)
          gf[i].v = *reinterpret_cast<const bf16x8 *>(gl + (c32 * WG_SR + i) * WG_GW + 16 * wave + 8 * h);
        // walk the input rows: A[ci][r][16w + 8h + e + v] (LDS col; col 0 = global j0 - 5)
        const bf16 *arow = al + (c32 * WG_LR) * WG_AW + 16 * wave + 8 * h + v;
#pragma unroll
        for (int r = 0; r < WG_LR; ++r) {
          Frag8<bf16> af;
          __builtin_memcpy(&af.v, arow + r * WG_AW, 16);
#pragma unroll
          for (int u = 0; u < 11; ++u) {
            const int i = r - u;
            if (i >= 0 && i < WG_SR) gf[i].mma(af, acc[u]);
          }
        }
      }
  float *dst = partial + ((long)blockIdx.x * 4 + wave) * 11 * 64 * 16;
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; r += 4)
      *reinterpret_cast<f32x4 *>(dst + (u * 64 + lane) * 16 + r) = f32x4{acc[u][r], acc[u][r + 1], acc[u][r + 2], acc[u][r + 3]};
}

// dW[co][ci][u][v] = sum over chunks and waves of the partials (fixed order).
__global__ void conv_wgrad_mid_reduce_kernel(const float *__restrict__ partial, float *__restrict__ dw, int CIN,
                                             int nchunk) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)32 * CIN * 121) return;
  const int v = (int)(idx % 11), u = (int)(idx / 11 % 11), ci = (int)(idx / 121 % CIN), co = (int)(idx / 121 / CIN);
  const int ct = ci >> 5;
  const int lane = 32 * ((co & 7) >> 2) + (ci & 31), r = 4 * (co >> 3) + (co & 3);
  float s = 0.0f;
  for (int c = 0; c < nchunk; ++c)
    for (int w = 0; w < 4; ++w)
      s += partial[((((long)(ct * 11 + v) * nchunk + c) * 4 + w) * 11 + u) * 64 * 16 + lane * 16 + r];
  dw[idx] = s;
}

size_t conv_wgrad_mid_partial_floats(int CIN, int nchunk) { return (size_t)(CIN / 32) * 11 * nchunk * 4 * 11 * 64 * 16; }

hipError_t conv_wgrad_mid(const bf16 *g, const bf16 *a, int CIN, float *partial, int nchunk, float *dw, int B,
                          int H, int W, hipStream_t s) {
  const int blocks = (CIN / 32) * 11 * nchunk;
  if (CIN == 64)
    conv_wgrad_mid_kernel<64><<<blocks, 256, 0, s>>>(g, a, partial, B, H, W, nchunk);
  else if (CIN == 32)
    conv_wgrad_mid_kernel<32><<<blocks, 256, 0, s>>>(g, a, partial, B, H, W, nchunk);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long n = (long)32 * CIN * 121;
  conv_wgrad_mid_reduce_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(partial, dw, CIN, nchunk);
  return hipGetLastError();
}

}  // namespace dsi

namespace dsi {

// ------------------------------------------------------------------------
// Weight gradient of the single-channel ends of the network (layer 1: one input
// channel; layer 3: one output channel) on MFMA.  With "wide" the tensor with
// 32k channels and "thin" the single-channel one, for filter row u:
//   THIN_OUT (layer 3): D_u[ci][v] = sum_{i,j'} a[ci][i+u-5][j'] * g[i][j'-v+5]
//   THIN_IN  (layer 1): D_u[co][v] = sum_{i,j}  g[co][i][j]      * x[i+u-5][j+v-5]
// M = wide channel (32 per tile), N = tap column v (11 of 32 used), K = 16
// columns; the thin operand is a Toeplitz band read with unaligned 16-byte
// LDS loads.  Layout and reduction as in conv_wgrad_mid_kernel.
constexpr int TG_PITCH = WG_TW + 16;  // thin tile pitch: cols -5 .. 74 (+ padding)

// wide [B][CW/16][H][W][16] (bf16); thin [B][H][W] (TT, converted to bf16)
// partial [ct*nchunk + chunk][4 waves][11 u][64 lanes][16] fp32
template <int MODE, typename TT>
__global__ __launch_bounds__(256) void conv_wgrad_thin_kernel(const bf16 *__restrict__ wide, const TT *__restrict__ thin,
                                                              int CW, float *__restrict__ partial, int B, int H, int W,
                                                              int nchunk) {
  constexpr int WR = MODE == THIN_OUT ? WG_LR : WG_SR;   // wide rows per strip
  constexpr int TR = MODE == THIN_OUT ? WG_SR : WG_LR;   // thin rows per strip
  __shared__ __attribute__((aligned(16))) bf16 wl[32 * WR * WG_GW];
  __shared__ __attribute__((aligned(16))) bf16 tl[TR * TG_PITCH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c32 = lane & 31;
  const int chunk = blockIdx.x % nchunk, ct = blockIdx.x / nchunk;
  const int per = (B + nchunk - 1) / nchunk;
  const int b0 = chunk * per, b1 = min(B, b0 + per);
  const int wrow0 = MODE == THIN_OUT ? -5 : 0, trow0 = MODE == THIN_OUT ? 0 : -5;

  f32x16 acc[11];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;

  for (int b = b0; b < b1; ++b)
    for (int i0 = 0; i0 < H; i0 += WG_SR)
      for (int j0 = 0; j0 < W; j0 += WG_TW) {
        __syncthreads();
        for (int idx = tid; idx < WR * WG_TW * 4; idx += 256) {
          const int q = idx & 3, pix = idx >> 2;
          const int row = pix / WG_TW, col = pix - row * WG_TW;
          const int gi = i0 + wrow0 + row, gj = j0 + col;
          const int c0 = ct * 32 + q * 8;
          bf16x8 val;
          if (gi >= 0 && gi < H && gj < W)
            val = *reinterpret_cast<const bf16x8 *>(wide + ((((long)b * (CW / 16) + (c0 >> 4)) * H + gi) * W + gj) * 16 + (c0 & 15));
          else
            for (int e = 0; e < 8; ++e) val[e] = (bf16)0.0f;
#pragma unroll
          for (int e = 0; e < 8; ++e) wl[((q * 8 + e) * WR + row) * WG_GW + col] = val[e];
        }
        for (int idx = tid; idx < TR * TG_PITCH; idx += 256) {
          const int row = idx / TG_PITCH, col = idx - row * TG_PITCH;
          const int gi = i0 + trow0 + row, gj = j0 - 5 + col;
          float val = 0.0f;
          if (gi >= 0 && gi < H && gj >= 0 && gj < W && col < WG_TW + 10) val = to_f32(thin[((long)b * H + gi) * W + gj]);
          tl[idx] = (bf16)val;
        }
        __syncthreads();
        const int j16 = 16 * wave + 8 * h;  // lane's 8 columns within the pass
        if constexpr (MODE == THIN_OUT) {
          // B_i[j'][v] = g[i][j' - v + 5]: thin LDS col (j' - v + 5) + 5 = j16 + e + 10 - v
          const int vv = c32 < 11 ? c32 : 0;
          Frag8<bf16> bf[WG_SR];
#pragma unroll
          for (int i = 0; i < WG_SR; ++i) {
            __builtin_memcpy(&bf[i].v, tl + i * TG_PITCH + j16 + 10 - vv, 16);
            if (c32 >= 11) bf[i] = frag_zero<bf16>();
          }
#pragma unroll
          for (int r = 0; r < WG_LR; ++r) {
            Frag8<bf16> af;
            af.v = *reinterpret_cast<const bf16x8 *>(wl + (c32 * WR + r) * WG_GW + j16);
#pragma unroll
            for (int u = 0; u < 11; ++u) {
              const int i = r - u;
              if (i >= 0 && i < WG_SR) af.mma(bf[i], acc[u]);
            }
          }
        } else {
          // A_i[co][j] = g[co][i][j]; B_r[j][v] = x[r][j + v - 5]: thin LDS col j16 + e + v
          const int vv = c32 < 11 ? c32 : 0;
          Frag8<bf16> af[WG_SR];
#pragma unroll
          for (int i = 0; i < WG_SR; ++i) af[i].v = *reinterpret_cast<const bf16x8 *>(wl + (c32 * WR + i) * WG_GW + j16);
#pragma unroll
          for (int r = 0; r < WG_LR; ++r) {
            Frag8<bf16> bfr;
            __builtin_memcpy(&bfr.v, tl + r * TG_PITCH + j16 + vv, 16);
            if (c32 >= 11) bfr = frag_zero<bf16>();
#pragma unroll
            for (int u = 0; u < 11; ++u) {
              const int i = r - u;
              if (i >= 0 && i < WG_SR) af[i].mma(bfr, acc[u]);
            }
          }
        }
      }
  float *dst = partial + ((long)blockIdx.x * 4 + wave) * 11 * 64 * 16;
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; r += 4)
      *reinterpret_cast<f32x4 *>(dst + (u * 64 + lane) * 16 + r) = f32x4{acc[u][r], acc[u][r + 1], acc[u][r + 2], acc[u][r + 3]};
}

// dW[m][u][v] (m = the wide channel; layer 3: [1][CW][11][11], layer 1: [CW][1][11][11]:
// the same linear order) = sum over chunks and waves of the partials.
__global__ void conv_wgrad_thin_reduce_kernel(const float *__restrict__ partial, float *__restrict__ dw, int CW,
                                              int nchunk) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= CW * 121) return;
  const int v = idx % 11, u = idx / 11 % 11, m = idx / 121;
  const int ct = m >> 5, ml = m & 31;
  const int lane = 32 * ((ml & 7) >> 2) + v, r = 4 * (ml >> 3) + (ml & 3);
  float s = 0.0f;
  for (int c = 0; c < nchunk; ++c)
    for (int w = 0; w < 4; ++w)
      s += partial[((((long)ct * nchunk + c) * 4 + w) * 11 + u) * 64 * 16 + lane * 16 + r];
  dw[idx] = s;
}

size_t conv_wgrad_thin_partial_floats(int CW, int nchunk) { return (size_t)(CW / 32) * nchunk * 4 * 11 * 64 * 16; }

template <typename TT>
hipError_t conv_wgrad_thin(int mode, const bf16 *wide, const TT *thin, int CW, float *partial, int nchunk, float *dw,
                           int B, int H, int W, hipStream_t s) {
  const int blocks = (CW / 32) * nchunk;
  if (mode == THIN_OUT)
    conv_wgrad_thin_kernel<THIN_OUT, TT><<<blocks, 256, 0, s>>>(wide, thin, CW, partial, B, H, W, nchunk);
  else
    conv_wgrad_thin_kernel<THIN_IN, TT><<<blocks, 256, 0, s>>>(wide, thin, CW, partial, B, H, W, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  conv_wgrad_thin_reduce_kernel<<<(CW * 121 + 255) / 256, 256, 0, s>>>(partial, dw, CW, nchunk);
  return hipGetLastError();
}

template hipError_t conv_wgrad_thin<float>(int, const bf16 *, const float *, int, float *, int, float *, int, int, int, hipStream_t);
template hipError_t conv_wgrad_thin<bf16>(int, const bf16 *, const bf16 *, int, float *, int, float *, int, int, int, hipStream_t);

}  // namespace dsi
