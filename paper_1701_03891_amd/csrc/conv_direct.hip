// conv_direct.hip -- direct (non-MFMA) kernels for Eq. (1) layers of ANY
// shape: channel counts C[l], odd filter sizes k[l].  They serve networks
// other than the paper's 1->64->32->1 11x11 stack (for which conv_mfma.hip
// has the fast kernels), the FP64 checking precision, and the backward pass.
//
// Eq. (1) per layer: z = corr(W, a) + b over the zero-padded input, the crop
// S keeping the centred n1 x n2 window ("same" correlation, padding (k-1)/2),
// then a = ReLU(z).  Activations are indexed through ActView so the same
// kernels read planar [B][C][H][W] or channel-blocked [B][C/16][H][W][16]
// tensors (the layout the MFMA kernels keep).
#include "common.h"
#include "internal.h"

namespace dsi {


template <typename Acc, typename T> DSI_INLINE Acc to_acc(T v) {
  if constexpr (sizeof(Acc) == 8 && sizeof(T) == 8) return v;
  else return (Acc)to_f32(v);
}
template <typename T> DSI_INLINE T from_acc(double v) { return from_f32<T>((float)v); }
template <> DSI_INLINE double from_acc<double>(double v) { return v; }
template <typename T> DSI_INLINE T from_acc(float v) { return from_f32<T>(v); }

// out(b,co,i,j) = act( sum_{ci,u,v} w[co][ci][u][v] in(b,ci,i+u-r,j+v-r) + bias )
template <typename TI, typename TW, typename TO, typename Acc>
__global__ __launch_bounds__(256) void conv_fwd_direct_kernel(const TI *__restrict__ in, ActView vi,
                                                              const TW *__restrict__ w,
                                                              const TW *__restrict__ bias, int bias_pp,
                                                              int relu, TO *__restrict__ out,
                                                              ActView vo, int k) {
  const int HW = vo.H * vo.W;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int co = blockIdx.y, b = blockIdx.z;
  const int i = p / vo.W, j = p % vo.W, r = (k - 1) / 2;
  Acc s = 0;
  for (int ci = 0; ci < vi.C; ++ci)
    for (int u = 0; u < k; ++u) {
      const int ii = i + u - r;
      if (ii < 0 || ii >= vi.H) continue;
      const TW *wr = w + (((long)co * vi.C + ci) * k + u) * k;
      for (int v = 0; v < k; ++v) {
        const int jj = j + v - r;
        if (jj < 0 || jj >= vi.W) continue;
        s += to_acc<Acc>(wr[v]) * to_acc<Acc>(in[act_idx(vi, b, ci, ii, jj)]);
      }
    }
  s += to_acc<Acc>(bias_pp ? bias[(long)co * HW + p] : bias[co]);
  if (relu && s < (Acc)0) s = 0;
  out[act_idx(vo, b, co, i, j)] = from_acc<TO>(s);
}

// Gradient with respect to the layer input, masked by the input's own ReLU:
// gin(b,ci,i,j) = [mask: a(b,ci,i,j) > 0] * sum_{co,u,v} gz(b,co,i-u+r,j-v+r) w[co][ci][u][v]
template <typename TG, typename TW, typename TA, typename TO, typename Acc>
__global__ __launch_bounds__(256) void conv_dgrad_direct_kernel(const TG *__restrict__ gz, ActView vg,
                                                                const TW *__restrict__ w,
                                                                const TA *__restrict__ amask,
                                                                ActView va, TO *__restrict__ gin,
                                                                ActView vo, int k) {
  const int HW = vo.H * vo.W;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int ci = blockIdx.y, b = blockIdx.z;
  const int i = p / vo.W, j = p % vo.W, r = (k - 1) / 2;
  if (amask && !(to_f32(amask[act_idx(va, b, ci, i, j)]) > 0.0f)) {
    gin[act_idx(vo, b, ci, i, j)] = from_acc<TO>((Acc)0);
    return;
  }
  Acc s = 0;
  for (int co = 0; co < vg.C; ++co)
    for (int u = 0; u < k; ++u) {
      const int ii = i - u + r;
      if (ii < 0 || ii >= vg.H) continue;
      const TW *wr = w + (((long)co * vo.C + ci) * k + u) * k;
      for (int v = 0; v < k; ++v) {
        const int jj = j - v + r;
        if (jj < 0 || jj >= vg.W) continue;
        s += to_acc<Acc>(gz[act_idx(vg, b, co, ii, jj)]) * to_acc<Acc>(wr[v]);
      }
    }
  gin[act_idx(vo, b, ci, i, j)] = from_acc<TO>(s);
}

// One block per weight (co, ci, u, v): dw = sum_{b,i,j} gz(b,co,i,j) in(b,ci,i+u-r,j+v-r),
// reduced in a fixed order (deterministic).
template <typename TG, typename TI, typename Acc, typename TD>
__global__ __launch_bounds__(256) void conv_wgrad_direct_kernel(const TG *__restrict__ gz, ActView vg,
                                                                const TI *__restrict__ in, ActView vi,
                                                                int B, int k, TD *__restrict__ dw) {
  __shared__ Acc red[256];
  const int widx = blockIdx.x;
  const int v = widx % k, u = (widx / k) % k, ci = (widx / (k * k)) % vi.C, co = widx / (k * k * vi.C);
  const int r = (k - 1) / 2, HW = vg.H * vg.W;
  Acc s = 0;
  for (long q = threadIdx.x; q < (long)B * HW; q += 256) {
    const int b = (int)(q / HW), p = (int)(q % HW);
    const int i = p / vg.W, j = p % vg.W, ii = i + u - r, jj = j + v - r;
    if (ii < 0 || ii >= vi.H || jj < 0 || jj >= vi.W) continue;
    s += to_acc<Acc>(gz[act_idx(vg, b, co, i, j)]) * to_acc<Acc>(in[act_idx(vi, b, ci, ii, jj)]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) dw[widx] = (TD)red[0];
}

// Bias gradient. Per pixel: db[co][p] = sum_b gz(b,co,p).  Per channel: one block per co.
template <typename TG, typename Acc, typename TD>
__global__ __launch_bounds__(256) void bias_grad_pp_kernel(const TG *__restrict__ gz, ActView vg, int B,
                                                           TD *__restrict__ db) {
  const int HW = vg.H * vg.W;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)vg.C * HW) return;
  const int co = (int)(idx / HW), p = (int)(idx % HW);
  Acc s = 0;
  for (int b = 0; b < B; ++b) s += to_acc<Acc>(gz[act_idx(vg, b, co, p / vg.W, p % vg.W)]);
  db[idx] = (TD)s;
}
template <typename TG, typename Acc, typename TD>
__global__ __launch_bounds__(256) void bias_grad_pc_kernel(const TG *__restrict__ gz, ActView vg, int B,
                                                           TD *__restrict__ db) {
  __shared__ Acc red[256];
  const int co = blockIdx.x, HW = vg.H * vg.W;
  Acc s = 0;
  for (long q = threadIdx.x; q < (long)B * HW; q += 256) {
    const int b = (int)(q / HW), p = (int)(q % HW);
    s += to_acc<Acc>(gz[act_idx(vg, b, co, p / vg.W, p % vg.W)]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = (TD)red[0];
}

// Per-pixel bias gradient over 16-byte units (EPU elements of TG): a block owns 16
// consecutive units of an image's tensor; its 16 thread groups each sum every 16th
// image of the batch, and the group sums are combined in group order (deterministic).
// Units are read contiguously whatever the layout: blocked [C/16][HW][16] (a unit is
// EPU channels of one pixel) or planar [C][HW] with HW % EPU == 0 (EPU pixels of one
// channel).
template <typename TG, typename TD>
__global__ __launch_bounds__(256) void bias_grad_units_kernel(const TG *__restrict__ gz, ActView vg, int B,
                                                              TD *__restrict__ db) {
  constexpr int EPU = 16 / (int)sizeof(TG);
  const int HW = vg.H * vg.W;
  const long NU = (long)vg.C * HW / EPU;
  const long u = (long)blockIdx.x * 16 + (threadIdx.x & 15);
  const int grp = threadIdx.x >> 4;
  float s[EPU];
#pragma unroll
  for (int e = 0; e < EPU; ++e) s[e] = 0.0f;
  if (u < NU) {
    for (int b = grp; b < B; b += 16) {
      const TG *src = gz + ((long)b * NU + u) * EPU;
      float x[EPU];
      if constexpr (sizeof(TG) == 2) {
        bf16x8 v = *reinterpret_cast<const bf16x8 *>(src);
#pragma unroll
        for (int e = 0; e < EPU; ++e) x[e] = (float)v[e];
      } else {
        f32x4 v = *reinterpret_cast<const f32x4 *>(src);
#pragma unroll
        for (int e = 0; e < EPU; ++e) x[e] = v[e];
      }
#pragma unroll
      for (int e = 0; e < EPU; ++e) s[e] += x[e];
    }
  }
  __shared__ float red[16][16][EPU];
#pragma unroll
  for (int e = 0; e < EPU; ++e) red[grp][threadIdx.x & 15][e] = s[e];
  __syncthreads();
  if (threadIdx.x >= 16 * EPU) return;
  const int ul = threadIdx.x / EPU, e = threadIdx.x % EPU;
  const long uu = (long)blockIdx.x * 16 + ul;
  if (uu >= NU) return;
  float t = 0.0f;
  for (int q = 0; q < 16; ++q) t += red[q][ul][e];
  long c, p;
  if (vg.blocked) {   // unit = (slice, pixel, part): channels slice*16 + part*EPU + e
    constexpr int UPP = 16 / EPU;   // units per pixel of a 16-channel slice
    const long cs = uu / ((long)HW * UPP), rem = uu % ((long)HW * UPP);
    p = rem / UPP;
    c = cs * 16 + (rem % UPP) * EPU + e;
  } else {            // unit = EPU consecutive pixels of one channel
    c = uu / (HW / EPU);
    p = (uu % (HW / EPU)) * EPU + e;
  }
  db[c * HW + p] = (TD)t;
}

// ------------------------------------------------------------------ launchers
template <typename TI, typename TW, typename TO, typename Acc>
hipError_t conv_fwd_direct(const TI *in, ActView vi, const TW *w, const TW *bias, int bias_pp,
                           int relu, TO *out, ActView vo, int B, int k, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  dim3 grid(ceil_div(vo.H * vo.W, 256), vo.C, B);
  conv_fwd_direct_kernel<TI, TW, TO, Acc><<<grid, 256, 0, s>>>(in, vi, w, bias, bias_pp, relu, out, vo, k);
  return hipGetLastError();
}
template <typename TG, typename TW, typename TA, typename TO, typename Acc>
hipError_t conv_dgrad_direct(const TG *gz, ActView vg, const TW *w, const TA *amask, ActView va,
                             TO *gin, ActView vo, int B, int k, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  dim3 grid(ceil_div(vo.H * vo.W, 256), vo.C, B);
  conv_dgrad_direct_kernel<TG, TW, TA, TO, Acc><<<grid, 256, 0, s>>>(gz, vg, w, amask, va, gin, vo, k);
  return hipGetLastError();
}
template <typename TG, typename TI, typename Acc, typename TD>
hipError_t conv_wgrad_direct(const TG *gz, ActView vg, const TI *in, ActView vi, int B, int k,
                             TD *dw, hipStream_t s) {
  const int nw = vg.C * vi.C * k * k;
  conv_wgrad_direct_kernel<TG, TI, Acc, TD><<<nw, 256, 0, s>>>(gz, vg, in, vi, B, k, dw);
  return hipGetLastError();
}
template <typename TG, typename Acc, typename TD>
hipError_t bias_grad(const TG *gz, ActView vg, int B, int per_pixel, TD *db, hipStream_t s) {
  constexpr int EPU = 16 / (int)sizeof(TG);
  const long HW = (long)vg.H * vg.W;
  const bool units = sizeof(Acc) == 4 && (vg.blocked ? (vg.C % 16 == 0) : (HW % EPU == 0));
  if (per_pixel && units) {
    const long nu = (long)vg.C * HW / EPU;
    bias_grad_units_kernel<TG, TD><<<(unsigned)((nu + 15) / 16), 256, 0, s>>>(gz, vg, B, db);
  } else if (per_pixel) {
    const long n = (long)vg.C * vg.H * vg.W;
    bias_grad_pp_kernel<TG, Acc, TD><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(gz, vg, B, db);
  } else {
    bias_grad_pc_kernel<TG, Acc, TD><<<vg.C, 256, 0, s>>>(gz, vg, B, db);
  }
  return hipGetLastError();
}

// explicit instantiations used by the host code
template hipError_t conv_fwd_direct<float, float, float, float>(const float *, ActView, const float *, const float *, int, int, float *, ActView, int, int, hipStream_t);
template hipError_t conv_fwd_direct<double, double, double, double>(const double *, ActView, const double *, const double *, int, int, double *, ActView, int, int, hipStream_t);

template hipError_t conv_dgrad_direct<float, float, float, float, float>(const float *, ActView, const float *, const float *, ActView, float *, ActView, int, int, hipStream_t);
template hipError_t conv_dgrad_direct<double, double, double, double, double>(const double *, ActView, const double *, const double *, ActView, double *, ActView, int, int, hipStream_t);
template hipError_t conv_dgrad_direct<float, float, bf16, float, float>(const float *, ActView, const float *, const bf16 *, ActView, float *, ActView, int, int, hipStream_t);

template hipError_t conv_wgrad_direct<float, float, float, float>(const float *, ActView, const float *, ActView, int, int, float *, hipStream_t);
template hipError_t conv_wgrad_direct<double, double, double, double>(const double *, ActView, const double *, ActView, int, int, double *, hipStream_t);
template hipError_t conv_wgrad_direct<float, bf16, float, float>(const float *, ActView, const bf16 *, ActView, int, int, float *, hipStream_t);

template hipError_t bias_grad<bf16, float, float>(const bf16 *, ActView, int, int, float *, hipStream_t);
template hipError_t bias_grad<float, float, float>(const float *, ActView, int, int, float *, hipStream_t);
template hipError_t bias_grad<double, double, double>(const double *, ActView, int, int, double *, hipStream_t);

}  // namespace dsi
