// gemm.hip -- the dense layers of the recovery path on MFMA.
//
//   measurement  y  = Phi x      : y[b][m]  = sum_n Phi[m][n]  x[b][n]   (Sec. 1)
//   proxy        x~ = Phi^T y    : x~[b][p] = sum_m Wfc[p][m]  y[b][m]   (Sec. 4)
//   proxy grad   dy = Wfc^T dx~  : dy[b][m] = sum_p WfcT[m][p] dx~[b][p]
//
// All three are C[b][o] = sum_k X[b][k] W[o][k] with both operands
// K-contiguous ("NT").  A wave owns a 32 (b) x 32 (o) tile of C; the four
// waves of a block cover 64 x 64.  MFMA A = X rows, B = W rows, so a lane
// holds C[b0 + row(r)][o0 + lane%32] and stores are 128-byte coalesced runs.
// The FC is HBM-bound below ~300 images per batch (W is streamed once per
// 32 images from L2) and MFMA-bound above.
#include "common.h"
#include "internal.h"

namespace dsi {

// 8 consecutive K values of row `row` starting at k (zero beyond K), as float.
template <typename TS>
DSI_INLINE void load8_checked(const TS *base, long ld, int row, int k, int K, float *out) {
  const TS *p = base + (long)row * ld + k;
#pragma unroll
  for (int e = 0; e < 8; ++e) out[e] = (k + e < K) ? to_f32(p[e]) : 0.0f;
}

// Raw 8-element operand as loaded (no conversion yet, so a prefetched load is
// not waited for until its k-step), then converted to the MFMA input type.
template <typename TS> struct Raw8;
template <> struct Raw8<bf16> {
  bf16x8 v;
  DSI_INLINE void ld(const bf16 *p) { v = *reinterpret_cast<const bf16x8 *>(p); }
};
template <> struct Raw8<float> {
  f32x4 a, b;
  DSI_INLINE void ld(const float *p) {
    a = *reinterpret_cast<const f32x4 *>(p);
    b = *reinterpret_cast<const f32x4 *>(p + 4);
  }
};
template <typename TM, typename TS> DSI_INLINE Frag8<TM> to_frag(const Raw8<TS> &r);
template <> DSI_INLINE Frag8<bf16> to_frag<bf16, bf16>(const Raw8<bf16> &r) {
  Frag8<bf16> f;
  f.v = r.v;
  return f;
}
template <> DSI_INLINE Frag8<float> to_frag<float, float>(const Raw8<float> &r) {
  Frag8<float> f;
  f.lo = r.a;
  f.hi = r.b;
  return f;
}
template <> DSI_INLINE Frag8<bf16> to_frag<bf16, float>(const Raw8<float> &r) {
  float x[8] = {r.a[0], r.a[1], r.a[2], r.a[3], r.b[0], r.b[1], r.b[2], r.b[3]};
  return frag_from<bf16>(x);
}
template <> DSI_INLINE Frag8<float> to_frag<float, bf16>(const Raw8<bf16> &r) {
  float x[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = (float)r.v[e];
  return frag_from<float>(x);
}

// C[b][o] = scale * sum_k X[b][k] W[o][k];  X [Bn][ldx] (TX), W [O][ldw] (TW), C [Bn][ldc] (TC).
// VEC: K % 16 == 0, ldx/ldw multiples of 8, pointers 16-byte aligned.
template <typename TX, typename TW, typename TC, typename TM, bool VEC>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const TX *__restrict__ X, long ldx,
                                                      const TW *__restrict__ W, long ldw,
                                                      TC *__restrict__ C, long ldc, int Bn, int O,
                                                      int K, float scale) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int o0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (b0 >= Bn || o0 >= O) return;
  const int rb = min(b0 + (lane & 31), Bn - 1);  // clamp rows: loads stay in bounds
  const int ro = min(o0 + (lane & 31), O - 1);
  const int kh = (lane >> 5) * 8;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  if constexpr (VEC) {
    // software pipeline: the operands of the next PF k-steps are in flight while
    // the current one multiplies (the loop is otherwise bound by L2 latency)
    constexpr int PF = 8;
    const TX *px = X + (long)rb * ldx + kh;
    const TW *pw = W + (long)ro * ldw + kh;
    const int nk = K / 16;
    Raw8<TX> rx[PF];
    Raw8<TW> rw[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p)
      if (p < nk) {
        rx[p].ld(px + p * 16);
        rw[p].ld(pw + p * 16);
      }
    for (int k = 0; k < nk; k += PF) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        if (k + p < nk) {
          const Frag8<TM> fx = to_frag<TM>(rx[p]), fw = to_frag<TM>(rw[p]);
          fx.mma(fw, acc);
          const int kn = k + p + PF;
          if (kn < nk) {
            rx[p].ld(px + kn * 16);
            rw[p].ld(pw + kn * 16);
          }
        }
      }
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 16) {
      float xs[8], ws[8];
      load8_checked(X, ldx, rb, k0 + kh, K, xs);
      load8_checked(W, ldw, ro, k0 + kh, K, ws);
      Frag8<TM> fx = frag_from<TM>(xs), fw = frag_from<TM>(ws);
      fx.mma(fw, acc);
    }
  }
  const int o = o0 + (lane & 31);
  if (o >= O) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = b0 + mfma_row(lane, r);
    if (b < Bn) C[(long)b * ldc + o] = from_f32<TC>(acc[r] * scale);
  }
}

// FP8 e4m3 variant: C[b][o] = oscale * sum_k Xq[b][k] Wq[o][k], both operands FP8 codes,
// rows padded with zero codes to K % 64 == 0 and 16-byte aligned; one 32x32x64
// MFMA per 64-wide K step (a lane holds 32 consecutive K codes).
__global__ __launch_bounds__(256) void gemm_nt_fp8_kernel(const u8 *__restrict__ X, long ldx, const u8 *__restrict__ W,
                                                          long ldw, bf16 *__restrict__ C, long ldc, int Bn, int O,
                                                          int K, float oscale) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int o0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (b0 >= Bn || o0 >= O) return;
  const int rb = min(b0 + (lane & 31), Bn - 1), ro = min(o0 + (lane & 31), O - 1);
  const int kh = (lane >> 5) * 32;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const u8 *px = X + (long)rb * ldx + kh, *pw = W + (long)ro * ldw + kh;
  constexpr int PF = 4;  // k-steps in flight
  const int nk = K / 64;
  Frag8<u8> fx[PF], fw[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < nk) {
      fx[p] = frag_load<u8>(px + p * 64);
      fw[p] = frag_load<u8>(pw + p * 64);
    }
  for (int k = 0; k < nk; k += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      if (k + p < nk) {
        fx[p].mma(fw[p], acc);
        const int kn = k + p + PF;
        if (kn < nk) {
          fx[p] = frag_load<u8>(px + kn * 64);
          fw[p] = frag_load<u8>(pw + kn * 64);
        }
      }
    }
  }
  const int o = o0 + (lane & 31);
  if (o >= O) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = b0 + mfma_row(lane, r);
    if (b < Bn) C[(long)b * ldc + o] = (bf16)(acc[r] * oscale);
  }
}

hipError_t gemm_nt_fp8(const u8 *X, long ldx, const u8 *W, long ldw, bf16 *C, long ldc, int Bn, int O, int K,
                       float oscale, hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  dim3 grid(ceil_div(O, 64), ceil_div(Bn, 64));
  gemm_nt_fp8_kernel<<<grid, 256, 0, s>>>(X, ldx, W, ldw, C, ldc, Bn, O, K, oscale);
  return hipGetLastError();
}

// Fragment-ordered operands (see pack_frag_*): a wave owns the 32 x 32 tile
// (bt, ot) and its k-step ks reads the contiguous fragments Xp[bt][ks] and
// Wp[ot][ks] (64 lanes x FE elements each), so every load instruction is one
// coalesced 1 KiB (bf16) or 2 KiB (FP8) run.  PF k-steps are kept in flight.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void gemm_frag_kernel(const T *__restrict__ Xp, const T *__restrict__ Wp,
                                                        TO *__restrict__ C, long ldc, int Bn, int O, int KS,
                                                        float scale) {
  constexpr int FE = sizeof(T) == 1 ? 32 : 8;
  constexpr int PF = sizeof(T) == 1 ? 8 : 16;   // k-steps in flight: the loads are latency-bound
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bt = blockIdx.y * 2 + (wave >> 1), ot = blockIdx.x * 2 + (wave & 1);
  if (bt * 32 >= Bn || ot * 32 >= O) return;
  const T *px = Xp + ((long)bt * KS * 64 + lane) * FE;
  const T *pw = Wp + ((long)ot * KS * 64 + lane) * FE;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  Frag8<T> fx[PF], fw[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int kp = min(p, KS - 1);
    fx[p] = frag_load<T>(px + (long)kp * 64 * FE);
    fw[p] = frag_load<T>(pw + (long)kp * 64 * FE);
  }
  // Full iterations of PF k-steps issue their loads unconditionally (past the end, of the
  // last k-step again), so each iteration has the same loads in flight and the wait before
  // a k-step's MFMA counts only the loads issued after its own (a conditional load or MFMA
  // would make the compiler wait for every load in flight at each iteration).  The last
  // KS mod PF k-steps were loaded by the last full iteration (or the prologue).
  const int KF = KS / PF * PF;
  for (int k = 0; k < KF; k += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      fx[p].mma(fw[p], acc);
      const int kn = min(k + p + PF, KS - 1);
      fx[p] = frag_load<T>(px + (long)kn * 64 * FE);
      fw[p] = frag_load<T>(pw + (long)kn * 64 * FE);
    }
  }
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < KS - KF) fx[p].mma(fw[p], acc);
  const int o = ot * 32 + (lane & 31);
  if (o >= O) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int b = bt * 32 + mfma_row(lane, r);
    if (b < Bn) C[(long)b * ldc + o] = (TO)(acc[r] * scale);
  }
}

hipError_t gemm_frag_bf16(const bf16 *Xp, const bf16 *Wp, bf16 *C, long ldc, int Bn, int O, int KS, hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  dim3 grid(ceil_div(O, 64), ceil_div(Bn, 64));
  gemm_frag_kernel<bf16, bf16><<<grid, 256, 0, s>>>(Xp, Wp, C, ldc, Bn, O, KS, 1.0f);
  return hipGetLastError();
}
hipError_t gemm_frag_bf16_f32(const bf16 *Xp, const bf16 *Wp, float *C, long ldc, int Bn, int O, int KS,
                              hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  dim3 grid(ceil_div(O, 64), ceil_div(Bn, 64));
  gemm_frag_kernel<bf16, float><<<grid, 256, 0, s>>>(Xp, Wp, C, ldc, Bn, O, KS, 1.0f);
  return hipGetLastError();
}
hipError_t gemm_frag_fp8(const u8 *Xp, const u8 *Wp, bf16 *C, long ldc, int Bn, int O, int KS, float scale,
                         hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  dim3 grid(ceil_div(O, 64), ceil_div(Bn, 64));
  gemm_frag_kernel<u8, bf16><<<grid, 256, 0, s>>>(Xp, Wp, C, ldc, Bn, O, KS, scale);
  return hipGetLastError();
}

// FP64 reference-precision variant (VALU), for the DSI_F64 checking path.
__global__ __launch_bounds__(256) void gemm_nt_f64_kernel(const double *__restrict__ X, long ldx,
                                                          const double *__restrict__ W, long ldw,
                                                          double *__restrict__ C, long ldc, int Bn,
                                                          int O, int K) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)Bn * O) return;
  const int b = (int)(idx / O), o = (int)(idx % O);
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += X[(long)b * ldx + k] * W[(long)o * ldw + k];
  C[(long)b * ldc + o] = s;
}

template <typename TX, typename TW, typename TC, typename TM>
hipError_t launch_gemm(const TX *X, long ldx, const TW *W, long ldw, TC *C, long ldc, int Bn, int O,
                       int K, bool vec, float scale, hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  dim3 grid(ceil_div(O, 64), ceil_div(Bn, 64));
  if (vec)
    gemm_nt_kernel<TX, TW, TC, TM, true><<<grid, 256, 0, s>>>(X, ldx, W, ldw, C, ldc, Bn, O, K, scale);
  else
    gemm_nt_kernel<TX, TW, TC, TM, false><<<grid, 256, 0, s>>>(X, ldx, W, ldw, C, ldc, Bn, O, K, scale);
  return hipGetLastError();
}

hipError_t gemm_nt_f32(const float *X, long ldx, const float *W, long ldw, float *C, long ldc,
                       int Bn, int O, int K, bool vec, hipStream_t s) {
  return launch_gemm<float, float, float, float>(X, ldx, W, ldw, C, ldc, Bn, O, K, vec, 1.0f, s);
}
hipError_t gemm_nt_bf16_out_bf16(const float *X, long ldx, const bf16 *W, long ldw, bf16 *C,
                                 long ldc, int Bn, int O, int K, bool vec, hipStream_t s) {
  return launch_gemm<float, bf16, bf16, bf16>(X, ldx, W, ldw, C, ldc, Bn, O, K, vec, 1.0f, s);
}
hipError_t gemm_nt_bf16_out_f32(const float *X, long ldx, const bf16 *W, long ldw, float *C,
                                long ldc, int Bn, int O, int K, bool vec, hipStream_t s) {
  return launch_gemm<float, bf16, float, bf16>(X, ldx, W, ldw, C, ldc, Bn, O, K, vec, 1.0f, s);
}
hipError_t gemm_nt_f64(const double *X, long ldx, const double *W, long ldw, double *C, long ldc,
                       int Bn, int O, int K, hipStream_t s) {
  if (Bn <= 0 || O <= 0) return hipSuccess;
  const long n = (long)Bn * O;
  gemm_nt_f64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(X, ldx, W, ldw, C, ldc, Bn, O, K);
  return hipGetLastError();
}

}  // namespace dsi
