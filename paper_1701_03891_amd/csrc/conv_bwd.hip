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
// the 18 A rows once, each A fragment (8 consecutive columns shifted by v - 5:
// the block stages its A strip already shifted by its tap column, so the read is
// a 16-byte aligned LDS load) feeding up to 8 MFMAs (one per u).
// Accumulators (11 u x 32 x 32) live across all strips and images of the
// block; each block then sums its four waves' accumulators in wave order and
// writes them, and a second kernel sums the blocks' partials in a fixed order
// (deterministic).  That blocked kernel serves widths W % 8 != 0; otherwise the
// activations and gradients are first copied channel-major and
// conv_wgrad_mid_vg_kernel (below) lets the four waves of a block share one staged
// strip across four tap columns.
#include "common.h"
#include "internal.h"

namespace dsi {

constexpr int WG_SR = 8;            // output rows per strip
constexpr int WG_LR = WG_SR + 10;   // input rows per strip
constexpr int WG_TW = 64;           // output columns per pass (4 waves x 16)
constexpr int WG_GW = WG_TW + 8;    // G tile row pitch (elements)
constexpr int WG_AW = WG_TW + 16;   // A tile row pitch (64 columns + padding)

// Sums the four waves' accumulators in wave order through LDS and stores the block's
// partial: per filter row u, the 1024 sums of the 32 x 32 tile as [r/4][lane][r%4]
// (THIN: only the 11 used band columns, 352 sums as [r/4][lane/32][lane%32 < 11][r%4]).
// red: 8192 floats of LDS that no wave still reads (the caller synchronises first).
template <bool THIN>
DSI_INLINE void store_block_partial(const f32x16 (&acc)[11], float *red, float *__restrict__ dst) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NQ = THIN ? 88 : 256;   // 4-float groups per u
  const int src = THIN ? (tid / 22) * 64 + ((tid / 11) & 1) * 32 + tid % 11 : tid;
#pragma unroll
  for (int u = 0; u < 11; ++u) {
    float *buf = red + (u & 1) * 4096;   // two buffers: one barrier per u
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4)
      *reinterpret_cast<f32x4 *>(buf + ((wave * 4 + r4) * 64 + lane) * 4) =
          f32x4{acc[u][4 * r4], acc[u][4 * r4 + 1], acc[u][4 * r4 + 2], acc[u][4 * r4 + 3]};
    __syncthreads();
    if (tid < NQ) {
      f32x4 t = *reinterpret_cast<const f32x4 *>(buf + src * 4);
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const f32x4 x = *reinterpret_cast<const f32x4 *>(buf + (w * 256 + src) * 4);
        t = f32x4{t[0] + x[0], t[1] + x[1], t[2] + x[2], t[3] + x[3]};
      }
      *reinterpret_cast<f32x4 *>(dst + (u * NQ + tid) * 4) = t;
    }
  }
}

// g [B][2][H][W][16] (T), a [B][CIN/16][H][W][16] (T)
// partial [(ct*11 + v)*nchunk + chunk][11 u][1024] fp32 (store_block_partial)
template <int CIN>
__global__ __launch_bounds__(256) void conv_wgrad_mid_kernel(const bf16 *__restrict__ g, const bf16 *__restrict__ a,
                                                             float *__restrict__ partial, int B, int H, int W,
                                                             int nchunk) {
  __shared__ __attribute__((aligned(16))) bf16 gl[32 * WG_SR * WG_GW];
  __shared__ __attribute__((aligned(16))) bf16 al[32 * WG_LR * WG_AW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c32 = lane & 31;
  // the (CIN/32) * 11 blocks of one image chunk read the same data: neighbours on one XCD
  const int L = xcd_logical(blockIdx.x, gridDim.x), ncombo = (CIN / 32) * 11;
  const int chunk = L / ncombo, v = (L % ncombo) % 11, ct = (L % ncombo) / 11;
  const int b0 = (int)((long)chunk * B / nchunk), b1 = (int)((long)(chunk + 1) * B / nchunk);  // balanced

  f32x16 acc[11];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;

  for (int b = b0; b < b1; ++b)
    for (int i0 = 0; i0 < H; i0 += WG_SR)
      for (int j0 = 0; j0 < W; j0 += WG_TW) {
        __syncthreads();
        // G strip: rows i0..i0+7, cols j0..j0+63, 32 channels (two 16-channel slices);
        // A strip: rows i0-5..i0+12, cols j0-5..j0+68, channels ct*32..ct*32+31.
        // Every load of a thread is issued before its (transposing) LDS stores.
        constexpr int NG = WG_SR * WG_TW * 4, NA = WG_LR * WG_TW * 4;
        constexpr int IG = (NG + 255) / 256, IA = (NA + 255) / 256, BA = 8;
        {
          i32x4 gv[IG];
#pragma unroll
          for (int it = 0; it < IG; ++it) {
            const int idx = tid + it * 256;
            const int q = idx & 3, pix = idx >> 2;               // q: 8-channel group
            const int row = pix / WG_TW, col = pix - row * WG_TW;
            const int gi = i0 + row, gj = j0 + col;
            gv[it] = i32x4{0, 0, 0, 0};
            if (idx < NG && gi < H && gj < W)
              gv[it] = *reinterpret_cast<const i32x4 *>(g + ((((long)b * 2 + (q >> 1)) * H + gi) * W + gj) * 16 + (q & 1) * 8);
          }
#pragma unroll
          for (int it = 0; it < IG; ++it) {
            const int idx = tid + it * 256;
            const int q = idx & 3, pix = idx >> 2;
            const int row = pix / WG_TW, col = pix - row * WG_TW;
            if (idx < NG) {
              bf16x8 e8;
              __builtin_memcpy(&e8, &gv[it], 16);
#pragma unroll
              for (int e = 0; e < 8; ++e) gl[((q * 8 + e) * WG_SR + row) * WG_GW + col] = e8[e];
            }
          }
        }
#pragma unroll 1
        for (int i0a = 0; i0a < IA; i0a += BA) {
          i32x4 av[BA];
#pragma unroll
          for (int j = 0; j < BA; ++j) {
            const int idx = tid + (i0a + j) * 256;
            const int q = idx & 3, pix = idx >> 2;
            const int row = pix / WG_TW, col = pix - row * WG_TW;
            const int gi = i0 - 5 + row, gj = j0 + v - 5 + col;
            const int c0 = ct * 32 + q * 8;
            av[j] = i32x4{0, 0, 0, 0};
            if (i0a + j < IA && idx < NA && gi >= 0 && gi < H && gj >= 0 && gj < W)
              av[j] = *reinterpret_cast<const i32x4 *>(a + ((((long)b * (CIN / 16) + (c0 >> 4)) * H + gi) * W + gj) * 16 + (c0 & 15));
          }
#pragma unroll
          for (int j = 0; j < BA; ++j) {
            const int idx = tid + (i0a + j) * 256;
            const int q = idx & 3, pix = idx >> 2;
            const int row = pix / WG_TW, col = pix - row * WG_TW;
            if (i0a + j < IA && idx < NA) {
              bf16x8 e8;
              __builtin_memcpy(&e8, &av[j], 16);
#pragma unroll
              for (int e = 0; e < 8; ++e) al[((q * 8 + e) * WG_LR + row) * WG_AW + col] = e8[e];
            }
          }
        }
        __syncthreads();
        // G fragments of the strip: lane (co = c32, h) holds G[co][i][16w + 8h + e]
        Frag8<bf16> gf[WG_SR];
#pragma unroll
        for (int i = 0; i < WG_SR; ++i)
          gf[i].v = *reinterpret_cast<const bf16x8 *>(gl + (c32 * WG_SR + i) * WG_GW + 16 * wave + 8 * h);
        // walk the input rows: A[ci][r][j0 + 16w + 8h + e + v - 5] (LDS col 0 = global j0 + v - 5,
        // so each fragment read is a 16-byte aligned LDS load)
        const bf16 *arow = al + (c32 * WG_LR) * WG_AW + 16 * wave + 8 * h;
#pragma unroll
        for (int r = 0; r < WG_LR; ++r) {
          Frag8<bf16> af;
          af.v = *reinterpret_cast<const bf16x8 *>(arow + r * WG_AW);
#pragma unroll
          for (int u = 0; u < 11; ++u) {
            const int i = r - u;
            if (i >= 0 && i < WG_SR) gf[i].mma(af, acc[u]);
          }
        }
      }
  __syncthreads();
  store_block_partial<false>(acc, reinterpret_cast<float *>(al),
                             partial + ((long)(ct * 11 + v) * nchunk + chunk) * 11 * 1024);
}

// ------------------------------------------------------------------------
// Channel-major copies for the conv2 weight gradient: x [B][C/16][HW][16] ->
// [B][C][HW].  A block transposes 16 channels x 64 pixels through LDS, so both the
// reads (64 pixels x 32 bytes) and the writes (16 rows of 128 bytes) are contiguous.
__global__ __launch_bounds__(256) void to_planar_kernel(const bf16 *__restrict__ in, bf16 *__restrict__ out, int C,
                                                        int HW) {
  __shared__ bf16 t[16][64 + 2];
  const int nchunk = (HW + 63) / 64;
  const int chunk = blockIdx.x % nchunk, cs = (blockIdx.x / nchunk) % (C / 16), b = blockIdx.x / nchunk / (C / 16);
  const int p0 = chunk * 64, tid = threadIdx.x;
  {
    const int p = tid >> 2, q = tid & 3;   // pixel, 4-channel quarter
    bf16x4 v;
    for (int e = 0; e < 4; ++e) v[e] = (bf16)0.0f;
    if (p0 + p < HW) v = *reinterpret_cast<const bf16x4 *>(in + (((long)b * (C / 16) + cs) * HW + p0 + p) * 16 + 4 * q);
#pragma unroll
    for (int e = 0; e < 4; ++e) t[4 * q + e][p] = v[e];
  }
  __syncthreads();
  const int c = tid >> 4, k = tid & 15;    // channel, 4-pixel group
  const int p = p0 + 4 * k;
  bf16 *dst = out + ((long)b * C + cs * 16 + c) * HW + p;
  if (p + 3 < HW) {
    bf16x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = t[c][4 * k + e];
    *reinterpret_cast<bf16x4 *>(dst) = v;
  } else {
    for (int e = 0; e < 4 && p + e < HW; ++e) dst[e] = t[c][4 * k + e];
  }
}

hipError_t to_planar(const bf16 *in, bf16 *out, int B, int C, int HW, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const long blocks = (long)B * (C / 16) * ((HW + 63) / 64);
  to_planar_kernel<<<(unsigned)blocks, 256, 0, s>>>(in, out, C, HW);
  return hipGetLastError();
}

// buffer_load_dwordx4 ... lds: the LLVM intrinsic, declared by its name so that the
// host pass of the compiler sees an ordinary declaration.  rsrc is a raw buffer
// resource (base, byte size); each lane's 16 bytes at byte offset voffset go to LDS
// at dst + 16 * lane (dst: the wave's common LDS address), zeros when the offset lies
// outside the resource.
__device__ void llvm_buffer_load_lds(i32x4 rsrc, __attribute__((address_space(3))) void *lds, int size, int voffset,
                                     int soffset, int offset, int aux) __asm("llvm.amdgcn.raw.buffer.load.lds");
DSI_INLINE i32x4 buffer_rsrc(const void *base, int bytes) {
  const unsigned long p = reinterpret_cast<unsigned long>(base);
  // (word 3: the raw-buffer configuration of gfx9 parts)
  return i32x4{(int)(unsigned)p, (int)((unsigned)(p >> 32) & 0xffffu), bytes, 0x00020000};
}
DSI_INLINE void buffer_load_lds16(const i32x4 &rsrc, i32x4 *dst, int voffset) {
  llvm_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)dst, 16, voffset, 0, 0, 0);
}

// conv2 weight gradient by tap-column groups, from channel-major g [B][32][H][W] and
// a [B][CIN][H][W] (W % 8 == 0, CIN * H * W < 2^31, B * H * W < 2^31).  A block owns a
// 32-channel input tile ct, a group of four tap columns and a range of strips (8
// output rows x 64 activation columns, in (image, row strip, column strip) order).
// Its wave w computes tap column v = 4 vg + w over every column of the strip (the
// twelfth slot repeats v = 10 and stores nothing), so four tap columns share one
// staged strip:
//   dW[co][ci][u][v] = sum_{i,j'} G[co][i][j' - v + 5] A[ci][i + u - 5][j'].
// A strip sits in LDS as two 32-column halves: activations (18 rows: 16 in the main
// tile, 2 in a tail) and gradients (8 rows x 64 columns, j0 - 16 .. j0 + 47 around the
// half starting at j0).  Every byte arrives by direct-to-LDS loads
// (buffer_load_dwordx4 ... lds; one instruction moves one channel's 16 x 32 activations
// or 8 x 64 gradients), 18 per wave per half, one per walk step: while the waves compute
// on one half, the other half of the next strip is loaded, so a barrier (two per strip)
// waits only for loads issued at least 18 steps earlier.  The walk is 4 chunks x 18
// input rows; each step's activation fragment is read 6 steps ahead and feeds up to 8
// MFMAs (one per filter row u).  The gradient fragment of row i starts 21 - v elements
// into its window row, a 16-byte LDS read at a 2-byte boundary.  Positions outside the
// image read past the buffer resource, which yields zeros.  Each wave stores its tap column's partial sums;
// conv_wgrad_mid_reduce_kernel adds the chunks in a fixed order.
constexpr int WV_CS = 65;        // channel stride (16-byte units) of the main and gradient tiles
constexpr int WV_TS = 9;         // channel stride of the activation tail (rows 16 and 17)
constexpr int WV_TN = 8 * 64;    // tail capacity: eight load instructions
constexpr int WV_LA = 8;         // read-ahead of the activation fragments (steps)

template <int CIN>
__global__ __launch_bounds__(256) void conv_wgrad_mid_vg_kernel(const bf16 *__restrict__ g,
                                                                const bf16 *__restrict__ a,
                                                                float *__restrict__ partial, int B, int H, int W,
                                                                int nchunk) {
  // channel strides of 1040 and 144 bytes: the 32 lanes of a half-wave read 32 channels
  // of one (row, column), on distinct banks
  __shared__ __attribute__((aligned(16))) i32x4 am0[32 * WV_CS], am1[32 * WV_CS], at0[WV_TN], at1[WV_TN];
  __shared__ __attribute__((aligned(16))) i32x4 gg0[32 * WV_CS], gg1[32 * WV_CS];
  const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5, c32 = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NCOMBO = (CIN / 32) * 3;
  // the NCOMBO blocks of one strip range read the same strips: neighbours on one XCD
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int chunk = L / NCOMBO, combo = L % NCOMBO, ct = combo / 3, vg = combo % 3;
  const int vw = 4 * vg + wave, v = vw < 11 ? vw : 10;
  const int nrs = (H + 7) / 8, ncs = (W + 63) / 64;
  const int S = B * nrs * ncs;
  const int s0 = (int)((long)S * chunk / nchunk), s1 = (int)((long)S * (chunk + 1) / nchunk);
  const int HW = H * W;
  const bf16 *aimg0 = a + (long)ct * 32 * HW;

  // a lane's unit in each kind of load instruction (fixed for the kernel):
  //   main: row lane / 4 of 16, unit lane % 4; gradient: row lane / 8, unit lane % 8;
  //   tail instruction 2 wave + q: unit t = 64 (2 wave + q) + lane of [channel][9]
  const int rowA = lane >> 2, colA = 8 * (lane & 3), rowG = lane >> 3, colG = 8 * (lane & 7) - 16;
  int cT[2], rowT[2], colT[2];
  bool okT[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int t = 64 * (2 * wave + q) + lane, c = t / WV_TS, slot = t - c * WV_TS;
    okT[q] = c < 32 && slot < 8;
    cT[q] = okT[q] ? c : 0;
    rowT[q] = 16 + (slot >> 2);
    colT[q] = 8 * (slot & 3);
  }
  struct Strip { int b, i0, j0; };
  auto strip_at = [&](int s) {
    const int b = s / (nrs * ncs), rem = s - b * nrs * ncs, rs = rem / ncs;
    return Strip{b, rs * 8, (rem - rs * ncs) * 64};
  };
  // Buffer resources over one channel plane (main and gradient tiles) or the 32
  // channels (tail) of the strip's image, in bytes; a load at offset 2^31 lies outside
  // and writes zeros, which is how halo positions outside the image are filled.
  constexpr int OOB = (int)0x80000000u;
  auto rsrc = [&](const bf16 *base, int bytes) { return buffer_rsrc(base, bytes); };
  // per-lane byte offsets of the load jobs of half hs of strip sp (the same for every
  // channel of the main and gradient tiles)
  // (and the strip's first channel planes of this wave's jobs)
  struct Offs { int a, t0, t1, g; const bf16 *pa, *pt, *pg; };
  auto offsets = [&](const Strip &sp, int hs) {
    const int jh = sp.j0 + 32 * hs;
    Offs o;
    o.pt = aimg0 + (long)sp.b * CIN * HW;
    o.pa = o.pt + (long)(8 * wave) * HW;
    o.pg = g + ((long)sp.b * 32 + 8 * wave) * HW;
    {
      const int gi = sp.i0 - 5 + rowA, gj = jh + colA;
      o.a = ((gi >= 0) & (gi < H) & (gj < W)) ? 2 * (gi * W + gj) : OOB;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int gi = sp.i0 - 5 + rowT[q], gj = jh + colT[q];
      const int t = (okT[q] & (gi >= 0) & (gi < H) & (gj < W)) ? 2 * (cT[q] * HW + gi * W + gj) : OOB;
      if (q == 0) o.t0 = t; else o.t1 = t;
    }
    {
      const int gi = sp.i0 + rowG, gj = jh + colG;
      o.g = ((gi < H) & (gj >= 0) & (gj < W)) ? 2 * (gi * W + gj) : OOB;
    }
    return o;
  };
  // load job m (0..17) of a half (offsets o): 0..7 the activation main tile of
  // channels 8 wave .. 8 wave + 7, 8..9 the tail, 10..17 the gradient tile of the same
  // channels
  auto dma_job = [&](const Offs &o, int hs, int m) {
    if (m < 8)
      buffer_load_lds16(rsrc(o.pa + m * HW, 2 * HW), (hs ? am1 : am0) + (8 * wave + m) * WV_CS, o.a);
    else if (m < 10)
      buffer_load_lds16(rsrc(o.pt, 64 * HW), (hs ? at1 : at0) + 64 * (2 * wave + m - 8), m == 8 ? o.t0 : o.t1);
    else
      buffer_load_lds16(rsrc(o.pg + (m - 10) * HW, 2 * HW), (hs ? gg1 : gg0) + (8 * wave + m - 10) * WV_CS, o.g);
  };
  // fragments of chunk k (columns 16k .. 16k + 15 of the strip): activation row r and
  // gradient row i
  auto read_a = [&](int k, int r) {
    Frag8<bf16> f;
    const i32x4 x = r < 16 ? ((k < 2) ? am0 : am1)[c32 * WV_CS + r * 4 + 2 * (k & 1) + h]
                           : ((k < 2) ? at0 : at1)[c32 * WV_TS + (r - 16) * 4 + 2 * (k & 1) + h];
    __builtin_memcpy(&f.v, &x, 16);
    return f;
  };
  // (the gradient fragment of row i in chunk k starts 16 (k % 2) + 8h + 21 - v elements
  // into its window row: one 16-byte read at a 2-byte boundary, which measured faster
  // than two aligned reads shifted in registers)
  const int goff = 8 * h + 21 - v;
  auto read_g = [&](int k, int i) {
    const bf16 *p = reinterpret_cast<const bf16 *>((k < 2) ? gg0 : gg1) + c32 * WV_CS * 8 + i * 64 + 16 * (k & 1) + goff;
    Frag8<bf16> f;
    f.v = *reinterpret_cast<const bf16x8 *>(p);
    return f;
  };

  f32x16 acc[11];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;

  constexpr int NST = 4 * 18, LA = WV_LA, B1 = 35 - LA, B2 = 71 - LA;
  static_assert(NST % LA == 0, "the read-ahead ring wraps with the strip");
  static_assert(18 - LA <= B1 + 1 && B1 + 18 <= B2, "load windows overlap");
  Frag8<bf16> aq[LA], gq[8];
  if (s0 < s1) {
    const Strip sp = strip_at(s0);
    const Offs o0 = offsets(sp, 0), o1 = offsets(sp, 1);
#pragma unroll
    for (int m = 0; m < 18; ++m) dma_job(o0, 0, m);
#pragma unroll
    for (int m = 0; m < WV_LA; ++m) dma_job(o1, 1, m);   // (the rest at the walk's first steps)
    __builtin_amdgcn_s_waitcnt(0);   // (a barrier alone does not wait for these loads)
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      aq[q] = read_a(0, q);
      if (q < 8) gq[q] = read_g(0, q);
    }
  }
  for (int s = s0; s < s1; ++s) {
    // (the last strip loads itself again: the same bytes into buffers nothing reads)
    const Strip cur = strip_at(s), nxt = strip_at(s + 1 < s1 ? s + 1 : s);
    const Offs oc1 = offsets(cur, 1), on0 = offsets(nxt, 0), on1 = offsets(nxt, 1);
    static_for<NST>([&](auto stc) {
      constexpr int st = decltype(stc)::value, k = st / 18, r = st % 18;
      const Frag8<bf16> x = aq[st % LA];
#pragma unroll
      for (int u = 0; u < 11; ++u) {
        const int i = r - u;
        if (i >= 0 && i < 8) gq[i].mma(x, acc[u]);
      }
      {   // reads for step st + LA (past the end: the next strip's first steps)
        constexpr int n = (st + LA) % NST, nk = n / 18, nr = n % 18;
        aq[st % LA] = read_a(nk, nr);
        if constexpr (nr < 8) gq[nr] = read_g(nk, nr);
      }
      // one load a step: this strip's second half (jobs LA..17), the next strip's first
      // half after the first barrier and its second half (jobs 0..LA-1) after the second
      if constexpr (st < 18 - LA) dma_job(oc1, 1, st + LA);
      else if constexpr (st > B1 && st <= B1 + 18) dma_job(on0, 0, st - B1 - 1);
      else if constexpr (st > B2) dma_job(on1, 1, st - B2 - 1);
      // after step B1 every read of the first half has been issued (the last, for step
      // 35, in this step), after step B2 every read of the second half; the reads issued
      // after a barrier find the half it waited for
      if constexpr (st == B1 || st == B2) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
      }
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  if (vw < 11) {
    float *dst = partial + ((long)(ct * 11 + v) * nchunk + chunk) * 11 * 1024;
#pragma unroll
    for (int u = 0; u < 11; ++u)
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4)
        *reinterpret_cast<f32x4 *>(dst + ((u * 4 + r4) * 64 + lane) * 4) =
            f32x4{acc[u][4 * r4], acc[u][4 * r4 + 1], acc[u][4 * r4 + 2], acc[u][4 * r4 + 3]};
  }
}

// Partial-sum reduction: a block owns RED_SLOTS consecutive accumulator slots; its
// RED_PARTS thread groups each sum every RED_PARTS-th partial of a slot in order, and
// the group sums are added in group order, so the result is the same on every run.
constexpr int RED_SLOTS = 32, RED_PARTS = 8;
DSI_INLINE float reduce_parts(float s) {
  __shared__ float red[RED_PARTS][RED_SLOTS];
  const int slot = threadIdx.x % RED_SLOTS, part = threadIdx.x / RED_SLOTS;
  red[part][slot] = s;
  __syncthreads();
  float t = 0.0f;
  if (part == 0)
    for (int q = 0; q < RED_PARTS; ++q) t += red[q][slot];
  return t;
}

// dW[co][ci][u][v] = sum over chunks of the blocks' partials (fixed order).  Slots
// (u, q) of one (ci tile, tap column) group are consecutive partials, q = the
// [r/4][lane][r%4] position in the 32 x 32 tile.
__global__ __launch_bounds__(256) void conv_wgrad_mid_reduce_kernel(const float *__restrict__ partial,
                                                                    float *__restrict__ dw, int CIN, int nchunk) {
  const long idx = (long)blockIdx.x * RED_SLOTS + (threadIdx.x % RED_SLOTS);
  const int part = threadIdx.x / RED_SLOTS;
  const long nslot = (long)(CIN / 32) * 11 * 11 * 1024;
  const int slot = (int)(idx % (11 * 1024));   // (u, q)
  const int grp = (int)(idx / (11 * 1024));    // ct * 11 + v
  float s = 0.0f;
  if (idx < nslot) {
    const float *p = partial + (long)grp * nchunk * 11 * 1024 + slot;
    for (int c = part; c < nchunk; c += RED_PARTS) s += p[(long)c * 11 * 1024];
  }
  s = reduce_parts(s);
  if (part != 0 || idx >= nslot) return;
  const int u = slot / 1024, q = slot % 1024, lane = (q >> 2) & 63, r = (q >> 8) * 4 + (q & 3);
  const int v = grp % 11, ct = grp / 11;
  const int co = mfma_row(lane, r), ci = ct * 32 + (lane & 31);
  dw[(((long)co * CIN + ci) * 11 + u) * 11 + v] = s;
}

size_t conv_wgrad_mid_partial_floats(int CIN, int nchunk) { return (size_t)(CIN / 32) * 11 * nchunk * 11 * 1024; }

// nchunk: image chunks of the blocked kernel, strip ranges of the channel-major one (the
// partials are [(ct * 11 + v) * nchunk + chunk][11 u][1024] either way)
hipError_t conv_wgrad_mid(const bf16 *g, const bf16 *a, int CIN, float *partial, int nchunk, float *dw, int B,
                          int H, int W, hipStream_t s, bool planar) {
  const int blocks = (CIN / 32) * 11 * nchunk;
  if (planar && (W % 8 != 0 || (long)CIN * H * W >= (1L << 31) || (long)B * H * W >= (1L << 31)))
    return hipErrorInvalidValue;
  if (CIN == 64 && planar)
    conv_wgrad_mid_vg_kernel<64><<<(CIN / 32) * 3 * nchunk, 256, 0, s>>>(g, a, partial, B, H, W, nchunk);
  else if (CIN == 64)
    conv_wgrad_mid_kernel<64><<<blocks, 256, 0, s>>>(g, a, partial, B, H, W, nchunk);
  else if (CIN == 32 && !planar)
    conv_wgrad_mid_kernel<32><<<blocks, 256, 0, s>>>(g, a, partial, B, H, W, nchunk);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long n = (long)(CIN / 32) * 11 * 11 * 1024;
  conv_wgrad_mid_reduce_kernel<<<(unsigned)((n + RED_SLOTS - 1) / RED_SLOTS), RED_SLOTS * RED_PARTS, 0, s>>>(
      partial, dw, CIN, nchunk);
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
// columns; the thin operand is a Toeplitz band read as four 32-bit LDS words from
// one of two copies of its tile (the other shifted by one element).  Layout and
// reduction as in conv_wgrad_mid_kernel.
constexpr int TG_PITCH = WG_TW + 16;  // thin tile pitch: cols -5 .. 74 (+ padding)

// wide [B][CW/16][H][W][16] (bf16); thin [B][H][W] (TT, converted to bf16)
// partial [ct*nchunk + chunk][11 u][352] fp32 (store_block_partial)
template <int MODE, typename TT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == THIN_OUT ? 1 : 2))) void conv_wgrad_thin_kernel(const bf16 *__restrict__ wide, const TT *__restrict__ thin,
                                                              int CW, float *__restrict__ partial, int B, int H, int W,
                                                              int nchunk) {
  constexpr int WR = MODE == THIN_OUT ? WG_LR : WG_SR;   // wide rows per strip
  constexpr int TR = MODE == THIN_OUT ? WG_SR : WG_LR;   // thin rows per strip
  __shared__ __attribute__((aligned(16))) bf16 wl[32 * WR * WG_GW];
  // the thin tile twice: as staged, and shifted left by one element, so every 8-wide
  // read can start on a 4-byte boundary (LDS reads at 2-byte offsets stall); the
  // second copy sits 64 bytes off a multiple of the bank width from the first
  constexpr int TCOPY = TR * TG_PITCH + 32;
  __shared__ __attribute__((aligned(16))) bf16 tl[2 * TCOPY];
  auto thin_frag = [&](int row, int start) {
    const int odd = start & 1;
    const uint32_t *p = reinterpret_cast<const uint32_t *>(tl + odd * TCOPY + row * TG_PITCH + start - odd);
    uint32_t w4[4] = {p[0], p[1], p[2], p[3]};
    Frag8<bf16> f;
    __builtin_memcpy(&f.v, w4, 16);
    return f;
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c32 = lane & 31;
  const int chunk = blockIdx.x % nchunk, ct = blockIdx.x / nchunk;
  // a block owns a balanced range of strips (8 rows x 64 columns, in (image, row
  // strip, column strip) order)
  const int nrs = (H + WG_SR - 1) / WG_SR, ncs = (W + WG_TW - 1) / WG_TW;
  const int S = B * nrs * ncs;   // (B * H * W < 2^31)
  const int s0 = (int)((long)S * chunk / nchunk), s1 = (int)((long)S * (chunk + 1) / nchunk);
  const int wrow0 = MODE == THIN_OUT ? -5 : 0, trow0 = MODE == THIN_OUT ? 0 : -5;

  f32x16 acc[11];
#pragma unroll
  for (int u = 0; u < 11; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0f;

  // Staging.  The wide strip moves as 8 x 8 blocks (8 channels x 8 columns of one row):
  // a thread loads the block's 8 pixels (16 bytes of 8 channels each), transposes them
  // in registers and stores 8 rows of 8 columns as 16-byte LDS writes.  For layer 3
  // both tiles of the next strip are loaded into registers while this strip's MFMAs
  // run.
  constexpr int NBLK = WR * (WG_TW / 8) * 4, NB = (NBLK + 255) / 256;
  constexpr int NTU = TR * TG_PITCH, IT = (NTU + 255) / 256;
  i32x4 wv[NB][8];
  float tv[IT];
  auto strip_load = [&](int sidx) {
    const bool live = sidx < s1;
    const int b = live ? sidx / (nrs * ncs) : 0, rem = sidx - b * nrs * ncs;
    const int i0 = (rem / ncs) * WG_SR, j0 = (rem % ncs) * WG_TW;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int blk = tid + n * 256, q = blk & 3, cg = (blk >> 2) & 7, row = blk >> 5;
      const int gi = i0 + wrow0 + row, gj = j0 + 8 * cg, c0 = ct * 32 + q * 8;
      const bool ok = live && blk < NBLK && gi >= 0 && gi < H;
      const bf16 *src = wide + ((((long)b * (CW / 16) + (c0 >> 4)) * H + gi) * W + gj) * 16 + (c0 & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        wv[n][e] = i32x4{0, 0, 0, 0};
        if (ok && gj + e < W) wv[n][e] = *reinterpret_cast<const i32x4 *>(src + e * 16);
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * 256;
      const int row = idx / TG_PITCH, col = idx - row * TG_PITCH;
      const int gi = i0 + trow0 + row, gj = j0 - 5 + col;
      tv[it] = 0.0f;
      if (live && idx < NTU && gi >= 0 && gi < H && gj >= 0 && gj < W && col < WG_TW + 10)
        tv[it] = to_f32(thin[((long)b * H + gi) * W + gj]);
    }
  };
  auto strip_store = [&]() {
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int blk = tid + n * 256, q = blk & 3, cg = (blk >> 2) & 7, row = blk >> 5;
      if (blk < NBLK) {
        // channel 8q + c of pixels 8cg .. 8cg + 7: dword k holds pixels 2k, 2k + 1
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const unsigned sel = (c & 1) ? 0x07060302u : 0x05040100u;
          i32x4 o;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            o[k] = (int)__builtin_amdgcn_perm((unsigned)wv[n][2 * k + 1][c >> 1], (unsigned)wv[n][2 * k][c >> 1], sel);
          *reinterpret_cast<i32x4 *>(wl + ((q * 8 + c) * WR + row) * WG_GW + 8 * cg) = o;
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * 256;
      if (idx < NTU) {
        const bf16 e = (bf16)tv[it];
        const int col = idx % TG_PITCH;
        tl[idx] = e;
        if (col > 0) tl[TCOPY + idx - 1] = e;
        if (col == TG_PITCH - 1) tl[TCOPY + idx] = (bf16)0.0f;
      }
    }
  };
  // (layer 1's kernel keeps two waves per SIMD, which the registers of a prefetched
  // strip would not allow: it loads each strip at its start instead)
  constexpr bool PF = MODE == THIN_OUT;
  if constexpr (PF) strip_load(s0);
  for (int sidx = s0; sidx < s1; ++sidx) {
        __syncthreads();   // the previous strip's fragments have been read
        if constexpr (!PF) strip_load(sidx);
        strip_store();
        __syncthreads();
        if constexpr (PF) strip_load(sidx + 1);   // (past the range: zeros, nothing loaded)
        const int j16 = 16 * wave + 8 * h;  // lane's 8 columns within the pass
        if constexpr (MODE == THIN_OUT) {
          // B_i[j'][v] = g[i][j' - v + 5]: thin LDS col (j' - v + 5) + 5 = j16 + e + 10 - v
          const int vv = c32 < 11 ? c32 : 0;
          Frag8<bf16> bf[WG_SR];
#pragma unroll
          for (int i = 0; i < WG_SR; ++i) {
            bf[i] = thin_frag(i, j16 + 10 - vv);
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
            bfr = thin_frag(r, j16 + vv);
            if (c32 >= 11) bfr = frag_zero<bf16>();
#pragma unroll
            for (int u = 0; u < 11; ++u) {
              const int i = r - u;
              if (i >= 0 && i < WG_SR) af[i].mma(bfr, acc[u]);
            }
          }
        }
      }
  __syncthreads();
  store_block_partial<true>(acc, reinterpret_cast<float *>(wl), partial + (long)blockIdx.x * 11 * 352);
}

// dW[m][u][v] (m = the wide channel; layer 3: [1][CW][11][11], layer 1: [CW][1][11][11]:
// the same linear order) = sum over chunks of the blocks' partials (fixed order); a
// slot is (u, q) of one channel tile, q = the [r/4][lane/32][v][r%4] position.
__global__ __launch_bounds__(256) void conv_wgrad_thin_reduce_kernel(const float *__restrict__ partial,
                                                                     float *__restrict__ dw, int CW, int nchunk) {
  const int idx = blockIdx.x * RED_SLOTS + (threadIdx.x % RED_SLOTS);
  const int part = threadIdx.x / RED_SLOTS;
  const int nslot = (CW / 32) * 11 * 352;
  const int slot = idx % (11 * 352), ct = idx / (11 * 352);
  float s = 0.0f;
  if (idx < nslot) {
    // four interleaved sums (partials c, c + 8, c + 16, c + 24 of each group of 32), so
    // that four loads are in flight; the order is fixed, so the result is reproducible
    const long st = (long)RED_PARTS * 11 * 352;
    const float *q = partial + (long)ct * nchunk * 11 * 352 + slot + (long)part * 11 * 352;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int c = part;
    for (; c + 3 * RED_PARTS < nchunk; c += 4 * RED_PARTS, q += 4 * st) {
      s0 += q[0];
      s1 += q[st];
      s2 += q[2 * st];
      s3 += q[3 * st];
    }
    for (; c < nchunk; c += RED_PARTS, q += st) s0 += q[0];
    s = (s0 + s1) + (s2 + s3);
  }
  s = reduce_parts(s);
  if (part != 0 || idx >= nslot) return;
  const int u = slot / 352, t = (slot % 352) >> 2, e = slot & 3;
  const int r4 = t / 22, h = (t / 11) & 1, v = t % 11;
  const int m = ct * 32 + 8 * r4 + 4 * h + e;   // mfma_row(32 h + v, 4 r4 + e)
  dw[((long)m * 11 + u) * 11 + v] = s;
}

size_t conv_wgrad_thin_partial_floats(int CW, int nchunk) { return (size_t)(CW / 32) * nchunk * 11 * 352; }

template <typename TT>
hipError_t conv_wgrad_thin(int mode, const bf16 *wide, const TT *thin, int CW, float *partial, int nchunk, float *dw,
                           int B, int H, int W, hipStream_t s) {
  const int blocks = (CW / 32) * nchunk;
  if ((long)B * H * W >= (1L << 31)) return hipErrorInvalidValue;   // strip indices are 32-bit
  if (mode == THIN_OUT)
    conv_wgrad_thin_kernel<THIN_OUT, TT><<<blocks, 256, 0, s>>>(wide, thin, CW, partial, B, H, W, nchunk);
  else
    conv_wgrad_thin_kernel<THIN_IN, TT><<<blocks, 256, 0, s>>>(wide, thin, CW, partial, B, H, W, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  conv_wgrad_thin_reduce_kernel<<<((CW / 32) * 11 * 352 + RED_SLOTS - 1) / RED_SLOTS, RED_SLOTS * RED_PARTS, 0,
                                  s>>>(partial, dw, CW, nchunk);
  return hipGetLastError();
}

template hipError_t conv_wgrad_thin<float>(int, const bf16 *, const float *, int, float *, int, float *, int, int, int, hipStream_t);
template hipError_t conv_wgrad_thin<bf16>(int, const bf16 *, const bf16 *, int, float *, int, float *, int, int, int, hipStream_t);

}  // namespace dsi
