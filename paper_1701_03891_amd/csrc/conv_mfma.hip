// conv_mfma.hip -- Eq. (1) layers of the paper's network (Sec. 5: 1 -> 64 -> 32
// -> 1 channels, 11 x 11 filters) as implicit GEMMs on CDNA4 matrix cores.
//
// Activation layout in HBM: channel-blocked [B][C/16][H][W][16] ("16-channel
// slices"), so one slice of a tile is a dense 2-D block of 32-byte (bf16) or
// 64-byte (fp32) pixels.  Weights are pre-packed in MFMA fragment order, so a
// wave loads a 32 x 16 weight fragment as one coalesced 1 KiB (bf16) read.
//
// conv_mid  (Cin % 16 == 0 -> Cout 32 or 64): the hot loop.  A wave owns
//   ROWS output rows x 32 columns x Cout channels.  For each 16-channel slice
//   and horizontal tap v it keeps the 11 vertical-tap weight fragments in
//   registers and walks the ROWS+10 input rows of its halo once: every
//   activation fragment read from LDS feeds up to ROWS MFMAs (one per output
//   row it reaches), so LDS traffic is ~1/5 of a naive implicit GEMM.
//   MFMA: A = weights (32 out-channels x 16 in-channels), B = activations
//   (16 in-channels x 32 pixels), D = 32 out-channels x 32 pixels.
// conv_first (Cin = 1 -> 64): K = taps; one MFMA k-step per filter row u,
//   its 16 K slots holding taps v = 0..10 (5 zero slots), gathered from a
//   small LDS tile of the proxy image.
// conv_last  (Cin = 32 -> 1): one output channel, a banded-Toeplitz GEMM on
//   16x16 MFMAs (output rows as N, the weight band built by lane shifts).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace dsi {

constexpr int KT = 11;   // filter size of the paper's layers
constexpr int RAD = 5;   // (KT - 1) / 2

// ----------------------------------------------------------------- LDS helpers
// Slice tiles live in LDS as [row][chunk][col] 16-byte units, so the 32 lanes
// of a half-wave read 32 consecutive units (conflict-free).
template <typename T> DSI_INLINE Frag8<T> lds_frag(const unsigned char *base, int plane_bytes);
template <> DSI_INLINE Frag8<bf16> lds_frag<bf16>(const unsigned char *p, int) {
  Frag8<bf16> f;
  f.v = *reinterpret_cast<const bf16x8 *>(p);
  return f;
}
template <> DSI_INLINE Frag8<float> lds_frag<float>(const unsigned char *p, int plane) {
  Frag8<float> f;
  f.lo = *reinterpret_cast<const f32x4 *>(p);
  f.hi = *reinterpret_cast<const f32x4 *>(p + plane);
  return f;
}
template <> DSI_INLINE Frag8<u8> lds_frag<u8>(const unsigned char *p, int plane) {
  Frag8<u8> f;
  const i32x4 lo = *reinterpret_cast<const i32x4 *>(p), hi = *reinterpret_cast<const i32x4 *>(p + plane);
  f.v = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return f;
}

// channels per HBM slice of a blocked activation tensor: 16 (bf16, fp32) or 64 (fp8)
template <typename T> constexpr int slice_ch() { return sizeof(T) == 1 ? 64 : 16; }

template <typename TO> DSI_INLINE void store4(TO *dst, float a, float b, float c, float d);
template <> DSI_INLINE void store4<float>(float *dst, float a, float b, float c, float d) {
  *reinterpret_cast<f32x4 *>(dst) = f32x4{a, b, c, d};
}
// FP8: saturate to the e4m3 range, then the hardware round-to-nearest-even conversion
template <> DSI_INLINE void store4<u8>(u8 *dst, float a, float b, float c, float d) {
  auto sat = [](float v) { return fminf(fmaxf(v, -448.0f), 448.0f); };
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat(a), sat(b), 0, false);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(sat(c), sat(d), lo, true);
  *reinterpret_cast<int *>(dst) = w;
}
template <> DSI_INLINE void store4<bf16>(bf16 *dst, float a, float b, float c, float d) {
  bf16x4 v;
  v[0] = (bf16)a; v[1] = (bf16)b; v[2] = (bf16)c; v[3] = (bf16)d;
  *reinterpret_cast<bf16x4 *>(dst) = v;
}
// BF16 store with ReLU after the conversion: on the bit patterns, max(x, 0) as 16-bit
// integers is ReLU (negative values and -0 have the sign bit set); floor = 0 applies it,
// floor = -32768 (the smallest 16-bit integer) leaves the values as they are.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
DSI_INLINE i32x2 pack4_bf16_floor(float a, float b, float c, float d, s16x2 floor) {
  const s16x2 lo = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2{a, b}), bf16x2));
  const s16x2 hi = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2{c, d}), bf16x2));
  return i32x2{__builtin_bit_cast(int, __builtin_elementwise_max(lo, floor)),
               __builtin_bit_cast(int, __builtin_elementwise_max(hi, floor))};
}
DSI_INLINE void store4_bf16_floor(bf16 *dst, float a, float b, float c, float d, s16x2 floor) {
  const s16x2 lo = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2{a, b}), bf16x2));
  const s16x2 hi = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2{c, d}), bf16x2));
  *reinterpret_cast<i32x2 *>(dst) = i32x2{__builtin_bit_cast(int, __builtin_elementwise_max(lo, floor)),
                                          __builtin_bit_cast(int, __builtin_elementwise_max(hi, floor))};
}
template <typename T> DSI_INLINE void load4f(const T *src, float *o);
template <> DSI_INLINE void load4f<float>(const float *src, float *o) {
  f32x4 v = *reinterpret_cast<const f32x4 *>(src);
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
template <> DSI_INLINE void load4f<bf16>(const bf16 *src, float *o) {
  bf16x4 v = *reinterpret_cast<const bf16x4 *>(src);
  o[0] = (float)v[0]; o[1] = (float)v[1]; o[2] = (float)v[2]; o[3] = (float)v[3];
}

// ------------------------------------------------------------------ LDS staging
// Copies up to NU 16-byte units into LDS.  unit(idx, loff) returns the global
// address of unit idx (nullptr with loff set: outside the image, zero-filled;
// nullptr with loff untouched: no such unit) and sets its LDS byte offset.  A thread issues the loads of a whole batch of its units before it
// stores any of them, so their HBM/L2 latencies overlap instead of adding up.
// MAXB bounds the batch (registers held by the loads in flight).
template <int NU, int NT, int MAXB = 16, typename F>
DSI_INLINE void stage_units(unsigned char *lds, int tid, F unit) {
  constexpr int NIT = (NU + NT - 1) / NT;
  constexpr int NB = (NIT + MAXB - 1) / MAXB;        // batches
  constexpr int BATCH = (NIT + NB - 1) / NB;         // balanced batch size <= MAXB
#pragma unroll
  for (int b0 = 0; b0 < NIT; b0 += BATCH) {
    i32x4 v[BATCH];
    int lo[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int idx = tid + (b0 + j) * NT;
      v[j] = i32x4{0, 0, 0, 0};
      lo[j] = -1;
      if (b0 + j < NIT && idx < NU) {
        const void *g = unit(idx, lo[j]);
        if (g) v[j] = *reinterpret_cast<const i32x4 *>(g);
      }
    }
#pragma unroll
    for (int j = 0; j < BATCH; ++j)
      if (lo[j] >= 0) *reinterpret_cast<i32x4 *>(lds + lo[j]) = v[j];
  }
}

// ===================================================================== conv_mid
// in   [B][CIN/SC][H][W][SC]  (T; SC = 16 channels per slice, 64 for FP8)
// wp   [CIN/SC][11 v][11 u][COUT/32][64 lanes][FE]  (T; FE = 8, 32 for FP8): lane l holds
//      W[co = ct*32 + l%32][ci = cs*SC + (l/32)*FE + e][u][v]
// EPI_BIAS: out = ReLU?(oscale * acc + bias); bias per channel [COUT] or per pixel in fragment
//      order [H][W][COUT/32][2][4][4] (fp32): position (c, h, q, e) of a pixel holds channel
//      32c + 8q + 4h + e, so a lane's 16 values of one row are 64 contiguous bytes
// EPI_MASK: out = acc * (mask > 0), mask in the output layout (backward through ReLU)
// oscale dequantises FP8 products (weight scale x activation scale); 1 otherwise.
// A block has WAVES waves stacked vertically (WAVES * ROWS output rows x 32 columns).
// The weight fragments of tap column v + 1 are loaded while tap column v computes.
// ASYNC (BF16): two LDS slice buffers.  While slice cs computes, each thread loads its
// units of the next slice (this tile's cs+1, or the block's next tile's first), two per tap
// column right after that column's weight loads, and stores them into the other buffer one
// column later, when they have long arrived (loads retire in order, so no wait the
// compiler places reaches further back than a column); one barrier per slice.  The last
// tap column also loads the next slice's first weight column.  One block per CU runs every
// G-th tile (G = the grid); without ASYNC, one block per tile.
template <typename T, int CIN, int COUT, int ROWS, int WAVES, int EPI, typename TO, bool ASYNC>
__global__ __launch_bounds__(64 * WAVES) void conv_mid_kernel(const T *__restrict__ in, const T *__restrict__ wp,
                                                              const float *__restrict__ bias, int bias_pp, int relu,
                                                              const T *__restrict__ mask, TO *__restrict__ out,
                                                              int H, int W, int tiles_w, int tiles_per_img,
                                                              int ntiles, float oscale) {
  constexpr int NT = 64 * WAVES;
  constexpr int TH = WAVES * ROWS, TW = 32, LH = TH + 2 * RAD, LW = TW + 2 * RAD;
  constexpr int SC = slice_ch<T>();
  constexpr int CH16 = SC * (int)sizeof(T) / 16;  // 16-byte chunks per pixel per slice: bf16 2, fp32 4, fp8 4
  constexpr int FE = 16 * (CH16 / 2) / (int)sizeof(T);  // fragment elements per lane: 8, 8, 32
  constexpr int NCT = COUT / 32, NCS = CIN / SC;
  constexpr int PLANE = LW * 16;              // bytes between chunk planes of one LDS row
  static_assert(!ASYNC || sizeof(T) == 2, "prefetched staging is for 2-byte types");
  constexpr int NU = LH * CH16 * LW;          // 16-byte units of one slice
  constexpr int NPF = (NU + NT - 1) / NT;     // units per thread per slice
  constexpr int BUF = NU * 16;                // bytes of one slice buffer
  __shared__ __attribute__((aligned(16))) unsigned char lds[(ASYNC ? 2 : 1) * BUF];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, px = lane & 31;
  // A block runs tiles tl, tl + G, ... (G = the grid; one tile per block unless the grid
  // is smaller than the tile count).  The tiles of one image (whose halos overlap) sit on
  // one XCD, side by side in time.
  const int G = gridDim.x;
  int tl = xcd_logical(blockIdx.x, G);
  auto tile_at = [&](int t_, int &img_, int &bi0_, int &bj0_) {
    img_ = t_ / tiles_per_img;
    const int r_ = t_ % tiles_per_img;
    bi0_ = (r_ / tiles_w) * TH;
    bj0_ = (r_ % tiles_w) * TW;
  };
  int img, bi0, bj0;
  tile_at(tl, img, bi0, bj0);

  // unit k of this thread (u = k NT + tid, [row][chunk][col] order) of slice sl of the
  // tile at (timg, ti0, tj0), zero outside the image
  auto unit_load = [&](int timg, int ti0, int tj0, int sl, int k) -> i32x4 {
    const int u = k * NT + tid;
    const int row = u / (CH16 * LW), rem = u - row * (CH16 * LW);
    const int chunk = rem / LW, col = rem - chunk * LW;
    const int gi = ti0 - RAD + row, gj = tj0 - RAD + col;
    i32x4 val = {0, 0, 0, 0};
    if (k < NPF && u < NU && gi >= 0 && gi < H && gj >= 0 && gj < W)
      val = *reinterpret_cast<const i32x4 *>(in + (long)(timg * NCS + sl) * H * W * SC + ((long)gi * W + gj) * SC +
                                             chunk * 8);
    return val;
  };
  auto unit_store = [&](unsigned char *b, int k, const i32x4 &val) {
    if (k < NPF && k * NT + tid < NU) *reinterpret_cast<i32x4 *>(b + (k * NT + tid) * 16) = val;
  };
  if constexpr (ASYNC) {
    i32x4 pf[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) pf[k] = unit_load(img, bi0, bj0, 0, k);
#pragma unroll
    for (int k = 0; k < NPF; ++k) unit_store(lds, k, pf[k]);
    __syncthreads();
  }
  int gsl = 0;   // slices computed so far by this block: their buffers alternate
  // weight fragments of the current and the next tap column (with prefetching, the
  // last column of a slice loads the next slice's first, so they outlive a tile)
  Frag8<T> wf[KT][NCT], wn[KT][NCT];

  for (;;) {   // over the block's tiles (one pass without prefetching)
  tile_at(tl, img, bi0, bj0);
  // the block's next tile: its first slice is prefetched during this tile's last one
  const bool has_next = tl + G < ntiles;
  int nimg = img, ni0 = bi0, nj0 = bj0;
  if (has_next) tile_at(tl + G, nimg, ni0, nj0);

  // With prefetched staging the accumulators start from the bias, so the epilogue
  // issues no loads.  Every bias load is unconditional, so all of them are in flight
  // together (a load under a branch makes the compiler wait for it before the next):
  // a pixel outside the image reads pixel 0's biases, and its outputs are never stored.
  constexpr bool PREBIAS = ASYNC && EPI == EPI_BIAS;
  f32x16 acc[ROWS][NCT];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int gi = bi0 + wave * ROWS + i, gj = bj0 + px;
    const long pix = gi < H && gj < W ? (long)gi * W + gj : 0;
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 b4 = {0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (PREBIAS)
          b4 = *reinterpret_cast<const f32x4 *>(bias + (bias_pp ? pix * COUT + c * 32 + h * 16 + q * 4
                                                                : (long)(c * 32 + 8 * q + 4 * h)));
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][c][4 * q + e] = b4[e];
      }
  }

  for (int cs = 0; cs < NCS; ++cs) {
   if constexpr (!ASYNC) {
    __syncthreads();  // previous slice fully consumed
    const T *src = in + (long)(img * NCS + cs) * H * W * SC;
    // 16 consecutive threads store 16 consecutive pixels of one chunk plane (no LDS bank
    // conflicts); a wave reads whole pixels, so its global reads stay contiguous
    // (wider types keep fewer loads in flight: their weight fragments need the registers)
    stage_units<(LH * LW + 15) / 16 * 16 * CH16, NT, sizeof(T) == 4 ? 2 : 16>(lds, tid, [&](int idx, int &loff) -> const void * {
      const int chunk = (idx >> 4) % CH16, pix = (idx / (16 * CH16)) * 16 + (idx & 15);
      if (pix >= LH * LW) return nullptr;
      const int row = pix / LW, col = pix - row * LW;
      const int gi = bi0 - RAD + row, gj = bj0 - RAD + col;
      loff = (row * CH16 + chunk) * PLANE + col * 16;
      if (gi < 0 || gi >= H || gj < 0 || gj >= W) return nullptr;
      return src + ((long)gi * W + gj) * SC + chunk * (16 / (int)sizeof(T));
    });
    __syncthreads();
   }
    const unsigned char *buf = lds + (ASYNC ? (gsl & 1) * BUF : 0);
    const T *wcs = wp + (long)cs * KT * KT * NCT * 64 * FE + lane * FE;
    // (with prefetching, the previous slice's last column already loaded this slice's
    // first weight column into wf)
    if (!ASYNC || gsl == 0) {
#pragma unroll
      for (int u = 0; u < KT; ++u)
#pragma unroll
        for (int c = 0; c < NCT; ++c) wf[u][c] = frag_load<T>(wcs + (u * NCT + c) * 64 * FE);
    }
    unsigned char *nbuf = lds + ((gsl + 1) & 1) * BUF;  // next slice's buffer (ASYNC), unread now
    // the slice prefetched during this one: the tile's next, or the next tile's first
    const bool pf_any = cs + 1 < NCS || has_next;
    const int pf_img = cs + 1 < NCS ? img : nimg, pf_i0 = cs + 1 < NCS ? bi0 : ni0;
    const int pf_j0 = cs + 1 < NCS ? bj0 : nj0, pf_sl = cs + 1 < NCS ? cs + 1 : 0;
    i32x4 pa0 = {0, 0, 0, 0}, pa1 = {0, 0, 0, 0};     // units loaded one column ago
    int pk = -1;                                       // their first unit index
    const unsigned char *lrow0 = buf + (wave * ROWS * CH16 + h * (CH16 / 2)) * PLANE + px * 16;
    // The slice is one walk over (tap column v, input row rr) steps.  With prefetched
    // staging each step's LDS fragment is read LA steps ahead (across column ends), and a
    // scheduling barrier after every step keeps the reads there, so a read's latency is
    // covered by the MFMAs of the steps between (at the band's ends a step has only 1-7).
    constexpr int NR = ROWS + 2 * RAD, NS = KT * NR, LA = ASYNC ? 6 : 1;
    Frag8<T> xq[LA];
    if constexpr (ASYNC) {
#pragma unroll
      for (int q = 0; q < LA; ++q) xq[q] = lds_frag<T>(lrow0 + (q / NR) * 16 + (q % NR) * CH16 * PLANE, PLANE);
    }
    // (unrolled when prefetching: every load then sits in straight-line code, and the
    // waits the compiler places for a column's weights count exactly the later loads)
#pragma unroll (ASYNC ? KT : 1)
    for (int v = 0; v < KT; ++v) {
      if (v + 1 < KT) {
#pragma unroll
        for (int u = 0; u < KT; ++u)
#pragma unroll
          for (int c = 0; c < NCT; ++c) wn[u][c] = frag_load<T>(wcs + (((v + 1) * KT + u) * NCT + c) * 64 * FE);
      } else if (ASYNC && pf_any) {   // the next slice's first column
        const T *wnx = wp + (long)pf_sl * KT * KT * NCT * 64 * FE + lane * FE;
#pragma unroll
        for (int u = 0; u < KT; ++u)
#pragma unroll
          for (int c = 0; c < NCT; ++c) wn[u][c] = frag_load<T>(wnx + (u * NCT + c) * 64 * FE);
      }
      if constexpr (ASYNC) {
        static_assert(NPF <= 2 * (KT - 1), "two units per column must cover the slice");
        if (pf_any) {
          if (pk >= 0) {
            unit_store(nbuf, pk, pa0);
            unit_store(nbuf, pk + 1, pa1);
          }
          pk = -1;
          if (2 * v < NPF) {
            pa0 = unit_load(pf_img, pf_i0, pf_j0, pf_sl, 2 * v);
            pa1 = unit_load(pf_img, pf_i0, pf_j0, pf_sl, 2 * v + 1);
            pk = 2 * v;
          }
        }
      }
      const unsigned char *lrow = lrow0 + v * 16;
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) {
        Frag8<T> xf;
        if constexpr (ASYNC) {
          const int st = v * NR + rr, q = st % LA, nx = st + LA;
          xf = xq[q];
          if (nx < NS) xq[q] = lds_frag<T>(lrow0 + (nx / NR) * 16 + (nx % NR) * CH16 * PLANE, PLANE);
        } else {
          xf = lds_frag<T>(lrow + rr * CH16 * PLANE, PLANE);
        }
#pragma unroll
        for (int u = 0; u < KT; ++u) {
          const int i = rr - u;  // output row (within the wave) that input row rr reaches through tap u
          if (i >= 0 && i < ROWS) {
#pragma unroll
            for (int c = 0; c < NCT; ++c) wf[u][c].mma(xf, acc[i][c]);
          }
        }
        if constexpr (ASYNC) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int u = 0; u < KT; ++u)
#pragma unroll
        for (int c = 0; c < NCT; ++c) wf[u][c] = wn[u][c];
    }
    if constexpr (ASYNC) {
      if (pf_any && pk >= 0) {
        unit_store(nbuf, pk, pa0);
        unit_store(nbuf, pk + 1, pa1);
      }
      __syncthreads();  // the next slice is in place and every wave is done with this one
    }
    ++gsl;
  }

  // epilogue: lane holds pixel (row i, col px), channels ct*32 + 8q + 4h + e
  const int gj = bj0 + px;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int gi = bi0 + wave * ROWS + i;
    if (gi >= H || gj >= W) continue;   // (the lanes px and px + 32 of a pixel together)
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      float vals[4][4];
      long o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int co0 = c * 32 + 8 * q + 4 * h;
        o[q] = ((((long)img * (COUT / 16) + (co0 >> 4)) * H + gi) * W + gj) * 16 + (co0 & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) vals[q][e] = acc[i][c][4 * q + e] * oscale;
        if constexpr (PREBIAS) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (relu) vals[q][e] = fmaxf(vals[q][e], 0.0f);
        } else if constexpr (EPI == EPI_BIAS) {
          float bv[4];
          if (bias_pp) load4f<float>(bias + ((long)gi * W + gj) * COUT + c * 32 + h * 16 + q * 4, bv);
          else load4f<float>(bias + co0, bv);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            vals[q][e] += bv[e];
            if (relu) vals[q][e] = fmaxf(vals[q][e], 0.0f);
          }
        } else {
          float mv[4];
          load4f<T>(mask + o[q], mv);
#pragma unroll
          for (int e = 0; e < 4; ++e) vals[q][e] = mv[e] > 0.0f ? vals[q][e] : 0.0f;
        }
      }
      if constexpr (sizeof(TO) == 2) {
        // lane h holds channels 4h.. (q even) and 8 + 4h.. (q odd) of a 16-channel slice;
        // one lane swap leaves it channels 8h .. 8h + 7, stored as one 16-byte unit
#pragma unroll
        for (int qp = 0; qp < 2; ++qp) {
          const s16x2 none = {-32768, -32768};
          i32x2 pa = pack4_bf16_floor(vals[2 * qp][0], vals[2 * qp][1], vals[2 * qp][2], vals[2 * qp][3], none);
          i32x2 pb = pack4_bf16_floor(vals[2 * qp + 1][0], vals[2 * qp + 1][1], vals[2 * qp + 1][2],
                                      vals[2 * qp + 1][3], none);
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const auto sw = __builtin_amdgcn_permlane32_swap((unsigned)pa[k], (unsigned)pb[k], false, false);
            pa[k] = (int)sw[0];
            pb[k] = (int)sw[1];
          }
          *reinterpret_cast<i32x4 *>(out + o[2 * qp] + 4 * h) = i32x4{pa[0], pa[1], pb[0], pb[1]};
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) store4<TO>(out + o[q], vals[q][0], vals[q][1], vals[q][2], vals[q][3]);
      }
    }
  }
  if constexpr (!ASYNC) break;
  tl += G;
  if (tl >= ntiles) break;
  }  // tiles
}

// =================================================================== conv_first
// One input channel -> COUT channels.  in [B][H][W] (TI, converted to T while
// staged), wp [11 u][COUT/32][64][8] (T): lane l holds
//     W[co = ct*32 + l%32][0][u][v = 8*(l/32) + e] (0 for v >= 11)
// out [B][COUT/16][H][W][16] (TO).
// A block owns a 4-row x 32-column tile of up to FIRST_IMGS images (one output
// row per wave) and stages all of their input halos in LDS at once.  Each wave
// keeps its bias values (and, for 2-byte types, all 11 x COUT/32 weight
// fragments) in registers across the images, so per image it only reads 11 LDS
// fragments, issues 11 x COUT/32 MFMAs and stores its row.
// The B operand of the k-step for filter row u is 8 consecutive pixels of one
// LDS row, read with one unaligned 16-byte LDS load.
// EPI_BIAS: out = ReLU?(acc + bias);  EPI_MASK: out = acc * (mask > 0).
// An FP8 output (TO = u8) is quantised as code = e4m3(oscale * value) into 64-channel slices.
constexpr int FIRST_IMGS = 16;

// Element-wise staging of conv_first's LDS tiles (any width, any input type): element
// (image im, row, col) of the tile is input pixel (r0 + row, c0 + col), zero outside;
// with two copies, the second holds each row shifted left by one element.
template <typename T, typename TI, int LH, int LWA, int NCOPY, int COPY>
DSI_INLINE void stage_first_scalar(T *tile, const TI *in, int tid, int nimg, int img0, int r0, int c0, int H, int W) {
  constexpr int NE = FIRST_IMGS * LH * LWA, NIT = (NE + 255) / 256, BATCH = 16;
  const int ne = nimg * LH * LWA;
#pragma unroll
  for (int b0 = 0; b0 < NIT; b0 += BATCH) {
    float v[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int idx = tid + (b0 + j) * 256;
      v[j] = 0.0f;
      if (b0 + j < NIT && idx < ne) {
        const int im = idx / (LH * LWA), rem = idx - im * (LH * LWA);
        const int row = rem / LWA, col = rem - row * LWA;
        const int gi = r0 + row, gj = c0 + col;
        if (gi >= 0 && gi < H && gj >= 0 && gj < W) v[j] = to_f32(in[((long)(img0 + im) * H + gi) * W + gj]);
      }
    }
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int idx = tid + (b0 + j) * 256;
      if (b0 + j < NIT && idx < ne) {
        const T e = from_f32<T>(v[j]);
        tile[idx] = e;
        if constexpr (NCOPY == 2) {
          const int col = idx % LWA;
          if (col > 0) tile[COPY + idx - 1] = e;
          if (col == LWA - 1) tile[COPY + idx] = from_f32<T>(0.0f);
        }
      }
    }
  }
}

template <typename T, int COUT, int EPI, typename TI, typename TO>
__global__ __launch_bounds__(256) void conv_first_kernel(const TI *__restrict__ in, const T *__restrict__ wp,
                                                         const float *__restrict__ bias, int bias_pp, int relu,
                                                         const T *__restrict__ mask, TO *__restrict__ out, int B,
                                                         int H, int W, int tiles_w, int tiles_per_img, int ipb,
                                                         float oscale) {
  constexpr int OSC = slice_ch<TO>();
  constexpr int TH = 4, TW = 32, LH = TH + 2 * RAD;
  // An LDS row holds input columns bj0 - 8 .. bj0 + 47 (OFF = 8 - RAD columns left of the
  // first tap): 16-byte aligned for vector staging, and wide enough for every 8-wide read.
  constexpr int OFF = 8 - RAD, LWA = 56, NVR = LWA / 8;
  constexpr int NCT = COUT / 32;
  constexpr bool WREG = sizeof(T) == 2;  // weights resident in registers
  // 2-byte types keep a second copy shifted by one element, so every 8-element read
  // starts on a 4-byte boundary (LDS reads at 2-byte offsets stall)
  constexpr int NCOPY = sizeof(T) == 2 ? 2 : 1;
  // (the copies sit 64 bytes off a multiple of the bank width apart, so the even and odd
  // lanes that read the same word index in the two copies use different banks)
  constexpr int COPY = FIRST_IMGS * LH * LWA + (NCOPY == 2 ? 32 : 0);
  __shared__ __attribute__((aligned(16))) T tile[NCOPY * COPY];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, px = lane & 31;
  const int grp = blockIdx.x / tiles_per_img, t = blockIdx.x % tiles_per_img;
  const int img0 = grp * ipb, nimg = min(ipb, B - img0);
  const int bi0 = (t / tiles_w) * TH, bj0 = (t % tiles_w) * TW;
  if constexpr (sizeof(TI) == 2 && sizeof(T) == 2) {
    if (W % 8 == 0) {
      // 16-byte vectors of 8 columns (all inside or all outside the image, as W % 8 == 0);
      // the shifted copy's vector is this vector and the next one funnel-shifted by one
      // element.  All loads of a thread are in flight before its LDS stores.
      constexpr int NV = FIRST_IMGS * LH * NVR, NIT = (NV + 255) / 256;
      const int nv = nimg * LH * NVR;
      i32x4 v[NIT], w[NIT];
#pragma unroll
      for (int j = 0; j < NIT; ++j) {
        const int idx = tid + j * 256;
        v[j] = w[j] = i32x4{0, 0, 0, 0};
        if (idx < nv) {
          const int im = idx / (LH * NVR), rem = idx - im * (LH * NVR);
          const int row = rem / NVR, vc = rem - row * NVR;
          const int gi = bi0 - RAD + row, gj = bj0 - 8 + 8 * vc;
          if (gi >= 0 && gi < H) {
            const TI *src = in + ((long)(img0 + im) * H + gi) * W;
            if (gj >= 0 && gj < W) v[j] = *reinterpret_cast<const i32x4 *>(src + gj);
            if (vc + 1 < NVR && gj + 8 >= 0 && gj + 8 < W) w[j] = *reinterpret_cast<const i32x4 *>(src + gj + 8);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NIT; ++j) {
        const int idx = tid + j * 256;
        if (idx < nv) {
          i32x4 sh;
          sh[0] = (int)__builtin_amdgcn_alignbit((unsigned)v[j][1], (unsigned)v[j][0], 16);
          sh[1] = (int)__builtin_amdgcn_alignbit((unsigned)v[j][2], (unsigned)v[j][1], 16);
          sh[2] = (int)__builtin_amdgcn_alignbit((unsigned)v[j][3], (unsigned)v[j][2], 16);
          sh[3] = (int)__builtin_amdgcn_alignbit((unsigned)w[j][0], (unsigned)v[j][3], 16);
          *reinterpret_cast<i32x4 *>(tile + idx * 8) = v[j];
          *reinterpret_cast<i32x4 *>(tile + COPY + idx * 8) = sh;
        }
      }
    } else {
      stage_first_scalar<T, TI, LH, LWA, NCOPY, COPY>(tile, in, tid, nimg, img0, bi0 - RAD, bj0 - 8, H, W);
    }
  } else {
    stage_first_scalar<T, TI, LH, LWA, NCOPY, COPY>(tile, in, tid, nimg, img0, bi0 - RAD, bj0 - 8, H, W);
  }

  const int gi = bi0 + wave, gj = bj0 + px;
  const bool live = gi < H && gj < W;
  float bv[NCT][4][4];
  if constexpr (EPI == EPI_BIAS) {
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int co0 = c * 32 + 8 * q + 4 * h;
        if (bias_pp) {  // planar [COUT][H][W]: consecutive lanes read consecutive pixels
#pragma unroll
          for (int e = 0; e < 4; ++e) bv[c][q][e] = live ? bias[((long)(co0 + e) * H + gi) * W + gj] : 0.0f;
        } else {
          load4f<float>(bias + co0, bv[c][q]);
        }
      }
  }
  Frag8<T> wr[WREG ? KT : 1][NCT];
  if constexpr (WREG) {
#pragma unroll
    for (int u = 0; u < KT; ++u)
#pragma unroll
      for (int c = 0; c < NCT; ++c) wr[u][c] = frag_load<T>(wp + ((u * NCT + c) * 64 + lane) * 8);
  }
  __syncthreads();

  // per-lane element offsets of the lane's 4-channel groups within one output image
  // (the same for the mask); images are img_stride elements apart
  const long img_stride = (long)(COUT / OSC) * H * W * OSC;
  const s16x2 floor = relu ? s16x2{0, 0} : s16x2{-32768, -32768};
  unsigned ooff[NCT][4];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co0 = c * 32 + 8 * q + 4 * h;
      ooff[c][q] = (unsigned)((((long)(co0 / OSC) * H + gi) * W + gj) * OSC + co0 % OSC);
    }
  // odd start column: read the shifted copy one element earlier (4-byte aligned)
  const int a0 = px + 8 * h + OFF, odd = NCOPY == 2 ? (a0 & 1) : 0;
  const T *trow0 = tile + odd * COPY + wave * LWA + a0 - odd;

  // 2-byte outputs and FP8 codes: an image's 16-byte stores per lane (four for BF16, two
  // for 64-channel FP8 pixels) are issued during the next image's MFMAs (then the last
  // image's after the loop), so the stores stream out between the matrix instructions
  // instead of stalling the wave in a burst; pend_off holds each one's element offset
  constexpr bool FP8OUT = sizeof(TO) == 1 && NCT == 2 && EPI == EPI_BIAS;
  constexpr bool PIPE = sizeof(TO) == 2 || FP8OUT;
  constexpr int NPEND = FP8OUT ? 2 : 2 * NCT;
  i32x4 pend[NPEND];
  unsigned pend_off[NPEND];
#pragma unroll
  for (int j = 0; j < NPEND; ++j)
    pend_off[j] = FP8OUT ? ooff[0][0] + 28 * h + 16 * j : ooff[j >> 1][2 * (j & 1)] + 4 * h;
  TO *pend_img = out;
  bool pend_live = false;
  for (int im = 0; im < nimg; ++im) {
    const long obase = (long)(img0 + im) * img_stride;   // uniform: the stores take it as a scalar base
    TO *const oimg = out + obase;
    float mv[NCT][4][4];
    if constexpr (EPI == EPI_MASK) {  // issued before the MFMAs so their latency overlaps
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (live) load4f<T>((mask + obase) + ooff[c][q], mv[c][q]);
    }
    f32x16 acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    // taps v = 8h + e of filter row u for output pixel px: LDS pixels px + 8h + e.  2-byte
    // types read each fragment as four 32-bit words (a 16-byte LDS read off a 16-byte
    // boundary stalls), all 11 issued before the MFMAs.  The slots of taps v >= 11 meet
    // zero weights, and every element read lies inside the staged (finite) tile row, so
    // they add exact zeros.
    const T *trow = trow0 + im * LH * LWA;
    uint32_t xw[KT][sizeof(Frag8<T>) / 4];
#pragma unroll
    for (int u = 0; u < KT; ++u) {
      const uint32_t *p32 = reinterpret_cast<const uint32_t *>(trow + u * LWA);
#pragma unroll
      for (int q = 0; q < (int)(sizeof(Frag8<T>) / 4); ++q) xw[u][q] = p32[q];
    }
#pragma unroll
    for (int u = 0; u < KT; ++u) {
      Frag8<T> xf;
      __builtin_memcpy(&xf, xw[u], sizeof(xf));
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        if constexpr (WREG) {
          wr[u][c].mma(xf, acc[c]);
        } else {
          const Frag8<T> wf = frag_load<T>(wp + ((u * NCT + c) * 64 + lane) * 8);
          wf.mma(xf, acc[c]);
        }
      }
      if constexpr (PIPE) {
        if (u >= 1 && u <= NPEND && pend_live) {
          const int j = u - 1;
          *reinterpret_cast<i32x4 *>(pend_img + pend_off[j]) = pend[j];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (PIPE) {
      pend_img = oimg;
      pend_live = live;
    }
    if (!live) continue;   // (the lanes px and px + 32 of a pixel are live together)
    if constexpr (sizeof(TO) == 2) {
      // Lane (px, h) holds channels 4h..4h+3 (q even) and 8+4h..11+4h (q odd) of each
      // 16-channel slice.  One swap of lanes 32..63 of the first group with lanes 0..31
      // of the second leaves lane h with channels 8h..8h+7, so each lane stores 16
      // bytes and a wave writes 32 whole pixels (1 KiB contiguous) per slice.
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int qp = 0; qp < 2; ++qp) {
          float va[4], vb[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            va[e] = acc[c][8 * qp + e];
            vb[e] = acc[c][8 * qp + 4 + e];
            if constexpr (EPI == EPI_BIAS) {
              va[e] += bv[c][2 * qp][e];
              vb[e] += bv[c][2 * qp + 1][e];
            } else {
              va[e] = mv[c][2 * qp][e] > 0.0f ? va[e] : 0.0f;
              vb[e] = mv[c][2 * qp + 1][e] > 0.0f ? vb[e] : 0.0f;
            }
          }
          const s16x2 fl = EPI == EPI_BIAS ? floor : s16x2{-32768, -32768};
          i32x2 pa = pack4_bf16_floor(va[0], va[1], va[2], va[3], fl);
          i32x2 pb = pack4_bf16_floor(vb[0], vb[1], vb[2], vb[3], fl);
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const auto sw = __builtin_amdgcn_permlane32_swap((unsigned)pa[k], (unsigned)pb[k], false, false);
            pa[k] = (int)sw[0];
            pb[k] = (int)sw[1];
          }
          // slice 2c + qp, channels 8h.. of the pixel: the q-even group's offset plus 4h
          // (stored during the next image's MFMAs)
          pend[2 * c + qp] = i32x4{pa[0], pa[1], pb[0], pb[1]};
        }
      continue;
    }
    if constexpr (sizeof(TO) == 1 && NCT == 2 && EPI == EPI_BIAS) {
      // FP8 codes, 64-channel pixels: lane (px, h) holds channels 32c + 8q + 4h .. +3.
      // Swapping lanes 32..63 of the c = 0 groups with lanes 0..31 of the c = 1 groups
      // leaves lane h with channels 32h .. 32h + 31: 32 bytes, two 16-byte stores.
      int code[2][4];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float vals[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            vals[e] = acc[c][4 * q + e] + bv[c][q][e];
            if (relu) vals[e] = fmaxf(vals[e], 0.0f);
            vals[e] = fminf(fmaxf(vals[e] * oscale, -448.0f), 448.0f);
          }
          const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(vals[0], vals[1], 0, false);
          code[c][q] = __builtin_amdgcn_cvt_pk_fp8_f32(vals[2], vals[3], lo, true);
        }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const auto sw = __builtin_amdgcn_permlane32_swap((unsigned)code[0][q], (unsigned)code[1][q], false, false);
        code[0][q] = (int)sw[0];
        code[1][q] = (int)sw[1];
      }
      // channel 32h of the pixel (ooff[0][0] points at 4h), stored during the next image's MFMAs
      pend[0] = i32x4{code[0][0], code[1][0], code[0][1], code[1][1]};
      pend[1] = i32x4{code[0][2], code[1][2], code[0][3], code[1][3]};
      continue;
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        TO *dst = oimg + ooff[c][q];
        float vals[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) vals[e] = acc[c][4 * q + e];
        if constexpr (EPI == EPI_BIAS) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            vals[e] += bv[c][q][e];
            if (relu) vals[e] = fmaxf(vals[e], 0.0f);
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) vals[e] = mv[c][q][e] > 0.0f ? vals[e] : 0.0f;
        }
        if constexpr (sizeof(TO) == 1) {
#pragma unroll
          for (int e = 0; e < 4; ++e) vals[e] *= oscale;
        }
        store4<TO>(dst, vals[0], vals[1], vals[2], vals[3]);
      }
  }
  if constexpr (PIPE) {   // the last image's stores
    if (pend_live) {
#pragma unroll
      for (int j = 0; j < NPEND; ++j) *reinterpret_cast<i32x4 *>(pend_img + pend_off[j]) = pend[j];
    }
  }
}

// ==================================================================== conv_last
// CIN channels -> one output channel.  BF16 uses conv_last_rows_kernel (further below);
// FP32 computes it as a banded-Toeplitz GEMM on 16x16 MFMAs:
// A wave owns 16 output rows x 16 output columns.  For horizontal tap v and
// each of the 26 input rows r of its halo:
//     D[j][i] += sum_c in[c][r][j + v - 5] * W[c][u = r - i][v]   (0 <= u <= 10)
// with M = output column j, N = output row i, K = input channels; the weight
// operand is the band of W for that (r, v), zero outside it.  Summing over
// r and v covers every (u, v) exactly once; 11/26 of the MFMA work is useful.
// in  [B][CIN/16][H][W][16] (T); wt [11 v][11 u][CIN] (T); out [B][H][W] fp32.
// Each pass over LDS holds 64 bytes of channels per pixel (32 bf16 / 16 fp32),
// as four 16-byte units; lane group g = l/16 reads unit g of its pixel.
template <typename T> DSI_INLINE void mma16(const Frag8<T> &a, const Frag8<T> &b, f32x4 &acc);

template <typename T, int CIN>
__global__ __launch_bounds__(256) void conv_last_kernel(const T *__restrict__ in, const T *__restrict__ wt,
                                                        const float *__restrict__ bias, int bias_pp, int relu,
                                                        float *__restrict__ out, int H, int W, int tiles_w,
                                                        int tiles_per_img) {
  constexpr int TH = 16, TW = 64, LH = TH + 2 * RAD, LW = TW + 2 * RAD;
  constexpr int EPU = 16 / (int)sizeof(T);   // elements per 16-byte unit
  constexpr int CHL = 4 * EPU;               // channels per pass
  constexpr int NPASS = CIN / CHL;
  constexpr int UNIT_PLANE = LW * 16;        // bytes between unit planes of one LDS row
  __shared__ __attribute__((aligned(16))) unsigned char lds[LH * 4 * UNIT_PLANE];
  __shared__ __attribute__((aligned(16))) T wl[KT * KT * CIN + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, n = lane & 15;
  // tiles of one image (whose halos overlap) on one XCD, side by side in time
  const int tl = xcd_logical(blockIdx.x, gridDim.x);
  const int img = tl / tiles_per_img, t = tl % tiles_per_img;
  const int bi0 = (t / tiles_w) * TH, bj0 = (t % tiles_w) * TW;
  {
    // weights as 16-byte units, every load issued before the stores
    constexpr int NWU = KT * KT * CIN / EPU, NIT = (NWU + 255) / 256;
    i32x4 wv[NIT];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int idx = tid + 256 * k;
      wv[k] = idx < NWU ? *reinterpret_cast<const i32x4 *>(wt + idx * EPU) : i32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k)
      if (tid + 256 * k < NWU) *reinterpret_cast<i32x4 *>(wl + (tid + 256 * k) * EPU) = wv[k];
  }
  f32x4 acc[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) acc[d] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int pass = 0; pass < NPASS; ++pass) {
    __syncthreads();
    // stage 16-byte units: unit q of pixel covers channels pass*CHL + q*EPU .. +EPU
    stage_units<(LH * LW + 15) / 16 * 16 * 4, 256>(lds, tid, [&](int idx, int &loff) -> const void * {
      const int q = (idx >> 4) & 3, pix = (idx >> 6) * 16 + (idx & 15);
      if (pix >= LH * LW) return nullptr;
      const int row = pix / LW, col = pix - row * LW;
      const int gi = bi0 - RAD + row, gj = bj0 - RAD + col;
      const int c0 = pass * CHL + q * EPU;
      loff = (row * 4 + q) * UNIT_PLANE + col * 16;
      if (gi < 0 || gi >= H || gj < 0 || gj >= W) return nullptr;
      return in + ((((long)img * (CIN / 16) + (c0 >> 4)) * H + gi) * W + gj) * 16 + (c0 & 15);
    });
    __syncthreads();
    // four tap columns at a time: four independent accumulator chains per row step
    for (int v0 = 0; v0 < KT; v0 += 4) {
      // Band operand B_r[n] = W[u = r - n][v] (zero outside 0..10).  Lane n at row r needs
      // what lane n-1 held at row r-1, so B_r is B_{r-1} shifted by one lane within each
      // 16-lane row (DPP row_shr:1, zero into lane 0), with lane 0 taking W[u = r].
      i32x4 band[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) band[d] = i32x4{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < LH; ++r) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int v = v0 + d;
          if (v < KT) {
            const unsigned char *arow = lds + g * UNIT_PLANE + (wave * 16 + n + v) * 16;
            Frag8<T> a, b;
            if constexpr (sizeof(T) == 2) {
              a.v = *reinterpret_cast<const bf16x8 *>(arow + r * 4 * UNIT_PLANE);
            } else {
              a.lo = *reinterpret_cast<const f32x4 *>(arow + r * 4 * UNIT_PLANE);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) band[d][q] = __builtin_amdgcn_update_dpp(0, band[d][q], 0x111, 0xf, 0xf, true);
            if (r < KT) {
              const i32x4 head = *reinterpret_cast<const i32x4 *>(wl + (v * KT + r) * CIN + pass * CHL + g * EPU);
              if (n == 0) band[d] = head;
            }
            __builtin_memcpy(&b, &band[d], 16);
            if constexpr (sizeof(T) == 4) b.hi = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            mma16<T>(a, b, acc[d]);
          }
        }
      }
    }
  }
  f32x4 accs = acc[0] + acc[1] + acc[2] + acc[3];
  // lane holds output row n, columns 4g .. 4g+3 of the wave's 16
  const int gi = bi0 + n;
  if (gi >= H) return;
  const int gj0 = bj0 + wave * 16 + 4 * g;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int gj = gj0 + e;
    if (gj >= W) break;
    float v = accs[e];
    if (bias) v += bias_pp ? bias[(long)gi * W + gj] : bias[0];
    out[((long)img * H + gi) * W + gj] = relu ? fmaxf(v, 0.0f) : v;
  }
}

template <> DSI_INLINE void mma16<bf16>(const Frag8<bf16> &a, const Frag8<bf16> &b, f32x4 &acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
}
template <> DSI_INLINE void mma16<float>(const Frag8<float> &a, const Frag8<float> &b, f32x4 &acc) {
#pragma unroll
  for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[e], b.lo[e], acc, 0, 0, 0);
}

// BF16 conv3 by rows: for each tap column v the partial sums over channels and filter
// rows, Q[i][j'][v] = sum_{c,u} W[c][u][v] a[c][i+u-5][j'], come from
// v_mfma_f32_16x16x32_bf16 with M = 16 input columns, N = v (11 of 16 used) and K = 32
// channels of one input row; the output is the column shift out[i][j] = sum_v
// Q[i][j+v-5][v] (+ bias).  A block owns 16 NWV input columns (16 NWV - 10 output columns)
// and a band of output rows of one image; wave w owns input columns 16w .. 16w + 15.
// A wave walks the input rows once: each row's activation fragment (lane: one pixel, 8
// consecutive channels: 16 bytes of the channel-blocked tensor) is loaded 11 rows ahead
// straight into registers and feeds 11 MFMAs, one per filter row u, into the accumulators
// of output rows r - u + 5 (11 rotating accumulators).  As output rows complete, the waves
// put their Q tiles in LDS; every RG rows, after one barrier, a thread per output adds its
// 11 shifted values and the bias (per-pixel biases staged in LDS once).
// WHOLE (images at most 16 NWV columns wide): the block's 16 NWV input columns are the
// whole image row, and it writes all of it.  The columns outside the image are zero, so
// their Q is zero: it is not computed, the Q rows in LDS carry 5 zero columns on either
// side instead, and no wave works on halo columns alone.
// in [B][CIN/16][H][W][16]; wt [11 v][11 u][CIN]; out [B][H][W].
template <int CIN, int NWV, int RB, bool WHOLE>
__global__ __launch_bounds__(64 * NWV) void conv_last_rows_kernel(const bf16 *__restrict__ in,
                                                                  const bf16 *__restrict__ wt,
                                                                  const float *__restrict__ bias, int bias_pp,
                                                                  int relu, float *__restrict__ out, int H, int W,
                                                                  int col_tiles, int row_tiles) {
  constexpr int NKS = CIN / 32, NIN = 16 * NWV, QS = 17, RG = 4;
  // Q columns held in LDS (index c: input column J0 - 5 + c) and output columns per block
  constexpr int NQ = WHOLE ? NIN + 10 : NIN, NOUT = NQ - 10, QOFF = WHOLE ? 5 : 0;
  static_assert(RG * NOUT <= 64 * NWV, "one thread per output of a row group");
  __shared__ float qs[2][RG][NQ * QS];
  __shared__ float bs[RB * NOUT];   // the block's per-pixel biases (loaded once)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, n16 = lane & 15;
  const int rt = blockIdx.x % row_tiles, ct = (blockIdx.x / row_tiles) % col_tiles;
  const int b = blockIdx.x / (row_tiles * col_tiles);
  const int I0 = rt * RB, I1 = min(I0 + RB, H), J0 = ct * NOUT;
  const int NR = I1 - I0 + 10;   // input rows I0 - 5 .. I1 + 4
  if constexpr (WHOLE) {   // the zero columns on either side (never written again)
    for (int idx = tid; idx < 2 * RG * 10 * QS; idx += 64 * NWV) {
      const int c = idx % (10 * QS), br = idx / (10 * QS);
      qs[br / RG][br % RG][c < 5 * QS ? c : (NQ - 10) * QS + c] = 0.0f;
    }
  }

  // B operands: lane (v = n16, channel group g) holds W[32 ks + 8g + e][u][v], zero for v = 11..15
  Frag8<bf16> wf[11][NKS];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      wf[u][ks] = frag_zero<bf16>();
      if (n16 < 11) wf[u][ks] = frag_load<bf16>(wt + (n16 * 11 + u) * CIN + 32 * ks + 8 * g);
    }
  // A operand source: input column j (M index n16), channels 32 ks + 8g .. + 7.  Rows come
  // through a buffer descriptor over this image, the lane's column in the vector offset and
  // the row in the scalar offset.  A vector offset of 2^31 (past the image, which the
  // launcher keeps under 2^31 bytes) reads as zeros, so rows and columns outside the image
  // take no branch, every row step issues the same loads, and the wait before a row's MFMAs
  // counts only the loads issued after it (a conditional load would make the compiler wait
  // for every load in flight once per pass over the ring).
  const int jc = J0 - 5 + QOFF + 16 * wave + n16;
  constexpr unsigned OOB = 0x80000000u;
  const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16 *>(in + (long)b * CIN * H * W), 0,
                                                      CIN * H * W * 2, 0x00020000);
  const unsigned lane_off =
      jc >= 0 && jc < W ? (unsigned)((((g >> 1) * H * W + jc) * 16 + 8 * (g & 1)) * 2) : OOB;
  auto a_load = [&](int t, int ks) {
    const int r = I0 - 5 + t;
    const bool rok = r >= 0 && r < H;
    Frag8<bf16> f;
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, rok ? lane_off : OOB, rok ? (2 * ks * H + r) * W * 32 : 0, 0);
    __builtin_memcpy(&f.v, &v, 16);
    return f;
  };
  Frag8<bf16> aq[11][NKS];
#pragma unroll
  for (int k = 0; k < 11; ++k)
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) aq[k][ks] = a_load(k, ks);
  f32x4 acc[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  // the reducing thread's row within a group of RG output rows, its output column
  const int rg = tid / NOUT, jt = tid - rg * NOUT, jo = J0 + jt;
  const bool io_ok = rg < RG && jo < W;
  const float b0 = bias && !bias_pp ? bias[0] : 0.0f;
  if (bias && bias_pp) {   // (read after the first reduction's barrier)
    for (int idx = tid; idx < RB * NOUT; idx += 64 * NWV) {
      const int r = idx / NOUT, c = idx - r * NOUT, i = I0 + r, j = J0 + c;
      bs[idx] = i < I1 && j < W ? bias[(long)i * W + j] : 0.0f;
    }
  }
  // one input row t in ring slot k = t mod 11; `load` refills the slot with row t + 11
  auto row = [&](auto kc, int t, bool load) {
    constexpr int k = decltype(kc)::value;
    // filter row u of input row t reaches output row I0 + t - u: its accumulator is
    // (k - u) mod 11, and u = 0 starts that row
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int u = 0; u < 11; ++u) {
        const int slot = (k - u + 11) % 11;
        const f32x4 c = (u == 0 && ks == 0) ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : acc[slot];
        acc[slot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[k][ks].v, wf[u][ks].v, c, 0, 0, 0);
      }
    if (load) {
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) aq[k][ks] = a_load(t + 11, ks);
    }
    if (t >= 10) {   // output row I0 + t - 10 is complete in accumulator (k + 1) mod 11
      constexpr int done = (k + 1) % 11;
      const int orow = t - 10, grp = orow / RG;
      float *q = qs[grp & 1][orow - grp * RG];
      // lane (v = n16, g) holds input columns 16 wave + 4g + e of tap column v
#pragma unroll
      for (int e = 0; e < 4; ++e) q[(QOFF + 16 * wave + 4 * g + e) * QS + n16] = acc[done][e];
      // every RG rows (and after the last) the threads add up the group's outputs
      if (orow - grp * RG == RG - 1 || t == NR - 1) {
        __syncthreads();
        const int i = I0 + grp * RG + rg;
        if (io_ok && i < I1) {
          const float *qr = qs[grp & 1][rg];
          float s = bias ? (bias_pp ? bs[(i - I0) * NOUT + jt] : b0) : 0.0f;
#pragma unroll
          for (int v = 0; v < 11; ++v) s += qr[(jt + v) * QS + v];
          out[((long)b * H + i) * W + jo] = relu ? fmaxf(s, 0.0f) : s;
        }
      }
    }
  };
  if constexpr (NKS == 1) {
    // full passes over the ring load the next pass's rows (past the band's end, unused
    // ones); the last NR mod 11 rows were loaded by the last full pass
    const int NF = NR / 11 * 11;
    for (int t0 = 0; t0 < NF; t0 += 11)
      static_for<11>([&](auto kc) { row(kc, t0 + decltype(kc)::value, true); });
    static_for<11>([&](auto kc) {
      if (NF + decltype(kc)::value < NR) row(kc, NF + decltype(kc)::value, false);
    });
  } else {
    // (64 channels: twice the fragments in registers; the one-body walk keeps them there)
    for (int t0 = 0; t0 < NR; t0 += 11)
      static_for<11>([&](auto kc) {
        const int t = t0 + decltype(kc)::value;
        if (t < NR) row(kc, t, t + 11 < NR);
      });
  }
}

// ==================================================================== launchers
// compute units of the current device (cached per device)
static int cu_count() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] <= 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}
static inline void tiles(int H, int W, int TH, int TW, int &tw, int &tpi) {
  tw = (W + TW - 1) / TW;
  tpi = tw * ((H + TH - 1) / TH);
}

template <typename T, int COUT, int EPI, typename TI, typename TO>
hipError_t conv_first(const TI *in, const T *wp, const float *bias, int bias_pp, int relu, const T *mask,
                      TO *out, int B, int H, int W, hipStream_t s, float oscale) {
  if (B <= 0) return hipSuccess;
  if ((long)COUT * H * W >= (1L << 31)) return hipErrorInvalidValue;   // per-image offsets are 32-bit
  int tw, tpi;
  tiles(H, W, 4, 32, tw, tpi);
  // images per block: enough blocks for two per CU, at most FIRST_IMGS
  const long want = ((long)B * tpi + 511) / 512;
  const int ipb = (int)std::max(1L, std::min((long)FIRST_IMGS, want));
  const int groups = (B + ipb - 1) / ipb;
  conv_first_kernel<T, COUT, EPI, TI, TO>
      <<<groups * tpi, 256, 0, s>>>(in, wp, bias, bias_pp, relu, mask, out, B, H, W, tw, tpi, ipb, oscale);
  return hipGetLastError();
}

template <typename T, int CIN, int COUT, int EPI, typename TO>
hipError_t conv_mid(const T *in, const T *wp, const float *bias, int bias_pp, int relu, const T *mask,
                    TO *out, int B, int H, int W, hipStream_t s, float oscale) {
  if (B <= 0) return hipSuccess;
  // BF16 with 32 outputs: 4 waves x 8 rows on a 32 x 32 tile, two 56 KiB slice buffers,
  // the next slice loaded into registers while this one computes.  BF16 with 64 outputs
  // (the data gradient of layer 2): 4 waves x 8 rows x 64 channels (256 accumulator
  // registers), one buffer.  FP32 and FP8: 4 waves, one buffer.
  constexpr int ROWS = COUT == 32 || sizeof(T) == 2 ? 8 : 4;
  constexpr int WAVES = 4;
  constexpr bool ASYNC = sizeof(T) == 2 && COUT == 32;
  int tw, tpi;
  tiles(H, W, WAVES * ROWS, 32, tw, tpi);
  const long ntiles = (long)B * tpi;
  if (ntiles >= (1L << 31)) return hipErrorInvalidValue;
  // prefetching kernel: one block per CU (its LDS allows no more), each running every
  // G-th tile and staging the next tile's first slice during its last; otherwise one
  // block per tile
  long grid = ntiles;
  if (ASYNC) grid = std::min(grid, (long)cu_count());
  conv_mid_kernel<T, CIN, COUT, ROWS, WAVES, EPI, TO, ASYNC><<<(unsigned)grid, 64 * WAVES, 0, s>>>(
      in, wp, bias, bias_pp, relu, mask, out, H, W, tw, tpi, (int)ntiles, oscale);
  return hipGetLastError();
}

template <typename T, int CIN>
hipError_t conv_last(const T *in, const T *w, const float *bias, int bias_pp, int relu, float *out, int B,
                     int H, int W, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 2) {
    // Images up to 64 (128) columns wide: 4 (8) waves over the whole row, one or two per
    // SIMD, bands of 32 output rows (with 4 waves two blocks share a CU).  Wider: 5 waves
    // over 80 input columns (70 outputs), bands of 64 rows.
    const int RB = W <= 128 ? 32 : 64;
    if ((long)CIN * H * W * 2 >= (1L << 31)) return hipErrorInvalidValue;   // buffer offsets are 31-bit
    const int row_tiles = (H + RB - 1) / RB;
    const int col_tiles = W <= 128 ? 1 : (W + 69) / 70;
    const long blocks = (long)B * col_tiles * row_tiles;
    if (blocks >= (1L << 31)) return hipErrorInvalidValue;
    if (W <= 64)
      conv_last_rows_kernel<CIN, 4, 32, true><<<(unsigned)blocks, 256, 0, s>>>(in, w, bias, bias_pp, relu, out, H, W,
                                                                            col_tiles, row_tiles);
    else if (W <= 128)
      conv_last_rows_kernel<CIN, 8, 32, true><<<(unsigned)blocks, 512, 0, s>>>(in, w, bias, bias_pp, relu, out, H, W,
                                                                            col_tiles, row_tiles);
    else
      conv_last_rows_kernel<CIN, 5, 64, false><<<(unsigned)blocks, 320, 0, s>>>(in, w, bias, bias_pp, relu, out, H,
                                                                             W, col_tiles, row_tiles);
  } else {
    int tw, tpi;
    tiles(H, W, 16, 64, tw, tpi);
    conv_last_kernel<T, CIN><<<B * tpi, 256, 0, s>>>(in, w, bias, bias_pp, relu, out, H, W, tw, tpi);
  }
  return hipGetLastError();
}

template hipError_t conv_first<bf16, 64, EPI_BIAS, bf16, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_first<float, 64, EPI_BIAS, float, float>(const float *, const float *, const float *, int, int, const float *, float *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<bf16, 64, 32, EPI_BIAS, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<float, 64, 32, EPI_BIAS, float>(const float *, const float *, const float *, int, int, const float *, float *, int, int, int, hipStream_t, float);
template hipError_t conv_first<bf16, 32, EPI_MASK, float, bf16>(const float *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_first<float, 32, EPI_MASK, float, float>(const float *, const float *, const float *, int, int, const float *, float *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<bf16, 32, 64, EPI_MASK, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<float, 32, 64, EPI_MASK, float>(const float *, const float *, const float *, int, int, const float *, float *, int, int, int, hipStream_t, float);
template hipError_t conv_last<bf16, 64>(const bf16 *, const bf16 *, const float *, int, int, float *, int, int, int, hipStream_t);
template hipError_t conv_last<float, 64>(const float *, const float *, const float *, int, int, float *, int, int, int, hipStream_t);
template hipError_t conv_first<bf16, 64, EPI_BIAS, bf16, u8>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, u8 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<u8, 64, 32, EPI_BIAS, bf16>(const u8 *, const u8 *, const float *, int, int, const u8 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_last<bf16, 32>(const bf16 *, const bf16 *, const float *, int, int, float *, int, int, int, hipStream_t);
// deeper or wider stacks of 11 x 11 layers with 32 or 64 hidden channels (BF16 recovery)
template hipError_t conv_first<bf16, 32, EPI_BIAS, bf16, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<bf16, 32, 32, EPI_BIAS, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<bf16, 32, 64, EPI_BIAS, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_mid<bf16, 64, 64, EPI_BIAS, bf16>(const bf16 *, const bf16 *, const float *, int, int, const bf16 *, bf16 *, int, int, int, hipStream_t, float);
template hipError_t conv_last<float, 32>(const float *, const float *, const float *, int, int, float *, int, int, int, hipStream_t);

}  // namespace dsi
