// Slice singular value thresholding (Sec. III-C, E-update), one complex
// h x w Fourier slice M per SliceDesc:
//
//   Ehat = M V diag(f) V^H   (h >= w, V = right singular vectors)
//   Ehat = U diag(f) U^H M   (h <  w, U = left singular vectors)
//   f_i  = max(1 - t / sigma_i, 0)
//
// Pipeline (one kernel each, all slices of all cubes batched):
//   k_gram       G = M^H M or M M^H (n1 x n1, packed lower triangle), MFMA,
//                FP32 or split-BF16 (3 terms) products
//   k_tridiag    Householder reduction G = Q T~ Q^H with Hermitian reflectors,
//                T~ Hermitian tridiagonal; made real by a diagonal phase;
//                the packed Gram stays in LDS when it fits
//   k_trieig     FP64 Sturm bisection for the eigenvalues above the
//                threshold and eigenvectors by twisted factorisations
//                (per unreduced block), cluster re-orthogonalisation
//   k_wy_t,      V <- Q (phase * z): the stored reflectors in blocks of 64
//   k_wy_apply   (compact WY form), applied with MFMA products
//   k_bp1        B = M V_r  (or U_r^H M), MFMA as the Gram
//   k_colnorm    sigma_i = ||M v_i|| (taken from M, not from the squared
//                Gram eigenvalue), f_i = max(1 - t/sigma_i, 0)
//   k_bp2        Ehat = B diag(f) V_r^H  (or U_r diag(f) B), written over M
//
// Eigenpairs whose Gram eigenvalue lies below t^2 - delta (delta a few FP32
// ulps of ||G||) are discarded: there sigma <= t and the shrink factor is 0.
#include "../../include/lrstv.h"
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"


namespace lrstv {

LRSTV_DEV int64_t packed(int r, int c) { return (int64_t)r * (r + 1) / 2 + c; }

// Deflation threshold of the Householder reduction: a column with
// ||x||^2 <= kDeflate2 (G scaled to ||G||_F ~ 1) is treated as zero.
#define kDeflate2 1e-14

// ------------------------------------------------------------------ Gram ---
// XCD-aware placement of a (tile, slice) grid launched as one dimension of
// ntile * round_up(ns, 8) blocks.  Workgroups are dispatched to the 8 XCDs
// in turn (block L to XCD L mod 8), each with its own L2; with slice =
// 8 (q / ntile) + L mod 8 and tile = q mod ntile (q = L / 8) the tiles of a
// slice run on one XCD at nearly the same time and share its L2.  Returns
// false for the padding slices.
LRSTV_DEV bool xcd_tile_slice(int ntile, int ns, int& tile, int& slice) {
  const int L = blockIdx.x, q = L >> 3, g = q / ntile;
  slice = 8 * g + (L & 7);
  tile = q - g * ntile;
  return slice < ns;
}
inline int xcd_grid(int ntile, int ns) { return ntile * ((ns + 7) / 8) * 8; }

// G = M^H M (tall) or M M^H (wide), packed lower triangle, one block per
// lower 64 x 64 tile (placed by xcd_tile_slice).
template <int MODE>
__global__ void __launch_bounds__(256) k_gram(const SliceDesc* __restrict__ desc, const float* __restrict__ sl,
                                              float2* __restrict__ gram, int ntile, int ns, const int* __restrict__ halt) {
  __shared__ MfmaSmem sm;
  int tile, slice;
  if (!xcd_tile_slice(ntile, ns, tile, slice)) return;
  const SliceDesc d = desc[slice];
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1, T = (n + kMT - 1) / kMT;
  int ti = 0, rem = tile;
  while (rem > ti) { rem -= ti + 1; ++ti; }
  const int tj = rem;
  if (ti >= T) return;
  const int h = d.h, w = d.w;
  const float* re = sl + d.a_off;
  const float* im = re + (int64_t)h * w;
  const int m0 = ti * kMT, n0 = tj * kMT;
  const int wv = threadIdx.x >> 6, r0 = m0 + 32 * (wv >> 1), c0 = n0 + 32 * (wv & 1);
  const bool active = r0 < n && c0 < n && r0 + 31 >= c0;
  float2* g = gram + d.g_off;
  // the diagonal of a Gram is real (its computed imaginary part is rounding)
  auto st = [&](int r, int c, float2 v) {
    if (r < n && c <= r) g[packed(r, c)] = r == c ? make_float2(v.x, 0.f) : v;
  };
  if (d.tall) {  // contraction over the h rows
    if constexpr (MODE == kF32) {
      // rows of M four columns at a time (float4 loads when aligned)
      auto row4 = [&](int k, int c, float sg, float2(&v)[4]) {
        const int nv = k < h ? n - c : 0;
        float a[4], b[4];
        load4(re + (int64_t)k * w + c, nv, a);
        load4(im + (int64_t)k * w + c, nv, b);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = make_float2(a[j], sg * b[j]);
      };
      auto fa = [&](int m, int k, float2(&v)[4]) { row4(k, m, -1.f, v); };
      auto fb = [&](int k, int c, float2(&v)[4]) { row4(k, c, 1.f, v); };
      mfma_ctile<MODE, false, false, true, true>(m0, n0, h, fa, fb, st, sm, active);
    } else {
      auto fa = [&](int m, int k) -> float2 {
        if (m >= n || k >= h) return make_float2(0.f, 0.f);
        const int64_t q = (int64_t)k * w + m;
        return make_float2(re[q], -im[q]);
      };
      auto fb = [&](int k, int c) -> float2 {
        if (c >= n || k >= h) return make_float2(0.f, 0.f);
        const int64_t q = (int64_t)k * w + c;
        return make_float2(re[q], im[q]);
      };
      mfma_ctile<MODE, false, false>(m0, n0, h, fa, fb, st, sm, active);
    }
  } else {  // contraction over the w columns
    auto fa = [&](int m, int k) -> float2 {
      if (m >= n || k >= w) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)m * w + k;
      return make_float2(re[q], im[q]);
    };
    auto fb = [&](int k, int c) -> float2 {
      if (c >= n || k >= w) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)c * w + k;
      return make_float2(re[q], -im[q]);
    };
    mfma_ctile<MODE, true, true>(m0, n0, w, fa, fb, st, sm, active);
  }
}

// Split-BF16 Gram on 128 x 128 tiles.  Each 32-wide k chunk of the tile's
// row and column operands is split once into hi / lo BF16 planes in LDS,
// and each wave computes a 64 x 64 block as 2 x 2 sub-tiles of
// v_mfma_f32_32x32x16_bf16, so that every fragment read from LDS feeds two
// products.  Products and terms as k_gram's split-BF16 mode.  A diagonal
// tile has one operand panel, staged once (two of the three tiles of a
// 256-wide slice).
//
// One block per CU (512 registers per lane), pipelined over the chunks:
// step c reads chunk c's fragments into registers, and after the barrier
// that frees the buffer issues the loads of chunk c + 2, splits chunk
// c + 1 (loaded during step c - 1) into the buffer and runs chunk c's
// products, the split and the products in one basic block so that the
// vector and LDS work issues between the products.
struct GramBfSmem {
  // planes 0 re hi, 1 re lo, 2 im hi, 3 im lo; row = the tile's row / column
  // index, the chunk's k contiguous (a lane's eight k are one 16-byte read)
  __bf16 a[4][128][kKC + kBfPad];
  __bf16 b[4][128][kKC + kBfPad];
};

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// hi = RNE_bf16(x) and lo = RNE_bf16(x - hi) (x - hi is exact in FP32) for a
// pair of values, each pair packed in one dword: one packed conversion per
// plane, the FP32 value of hi by a shift / mask of its bits.
LRSTV_DEV void bf_split2(float x0, float x1, unsigned& hi, unsigned& lo) {
  const f32x2v x = {x0, x1};
  const unsigned u = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2v));
  const f32x2v r = {x0 - __uint_as_float(u << 16), x1 - __uint_as_float(u & 0xffff0000u)};
  hi = u;
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2v));
}

// Split eight consecutive values (one k run of one row) into the four
// planes at row `row`, k offset k0 of the chunk.
LRSTV_DEV void bf_split_store(__bf16 (*p)[128][kKC + kBfPad], int row, int k0, const float (&re)[8],
                              const float (&im)[8]) {
  uint4 rh, rl, ih, il;
  bf_split2(re[0], re[1], rh.x, rl.x);
  bf_split2(re[2], re[3], rh.y, rl.y);
  bf_split2(re[4], re[5], rh.z, rl.z);
  bf_split2(re[6], re[7], rh.w, rl.w);
  bf_split2(im[0], im[1], ih.x, il.x);
  bf_split2(im[2], im[3], ih.y, il.y);
  bf_split2(im[4], im[5], ih.z, il.z);
  bf_split2(im[6], im[7], ih.w, il.w);
  *(uint4*)&p[0][row][k0] = rh;
  *(uint4*)&p[1][row][k0] = rl;
  *(uint4*)&p[2][row][k0] = ih;
  *(uint4*)&p[3][row][k0] = il;
}

// One thread's share of a chunk, 32 complex values.
struct BfChunk { float r[32], i[32]; };

// Chunk staging.  The planes hold Re M and Im M with no conjugation; an
// operand panel is 128 rows (indices of the Gram) by the chunk's 32 k.
//
// FAST (w a multiple of 4, K a multiple of the chunk width, 16-byte aligned
// planes): straight-line loads with clamped indices and no selects.  Rows
// or columns past n only reach Gram entries past n, which are not stored,
// and chunks past K are split into the buffer but never read, so the
// clamped loads may return any data there.  On a diagonal tile (DIAG) the
// two operands are one panel, staged once by all 256 threads (s = t);
// otherwise threads 0-127 stage the row operand and 128-255 the column
// operand (s = t mod 128).
//   tall (panel rows = columns of M, k = rows of M): a lane holds two
//     adjacent columns (float2 loads along a row of M) of DIAG ? 8 : 16
//     rows, v[2 r + c] = M(k0 + kb + r, col + c), so that the 16-byte LDS
//     stores of 16 lanes fall on distinct bank pairs (four columns per lane
//     would put them on one bank quarter);
//   wide (panel rows = rows of M, k contiguous): DIAG ? 2 : 4 runs of eight
//     k, v[8 u + j] = M(row_u, k0 + 8 q_u + j).
// Otherwise (SLOW) each load checks its range and reads zeros past it:
// tall, four columns of eight rows (v[4 r + c]); wide as FAST.
template <bool TALL, bool DIAG>
LRSTV_DEV void bf_fetch_fast(BfChunk& v, const float* re, const float* im, int h, int w, int n, int base, int s,
                             int k0) {
  const int K = TALL ? h : w, kc = min(k0, K - kKC);
  if (TALL) {
    constexpr int NR = DIAG ? 8 : 16;
    const int col = min(base + 2 * (s & 63), n - 2), r0 = kc + NR * (s >> 6);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t o = (int64_t)(r0 + r) * w + col;
      const float2 x = *reinterpret_cast<const float2*>(re + o), y = *reinterpret_cast<const float2*>(im + o);
      v.r[2 * r] = x.x; v.r[2 * r + 1] = x.y;
      v.i[2 * r] = y.x; v.i[2 * r + 1] = y.y;
    }
  } else {
    constexpr int NU = DIAG ? 2 : 4, STEP = DIAG ? 256 : 128;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = s + STEP * u, mr = min(base + (e >> 2), n - 1);
      const int64_t o = (int64_t)mr * w + kc + 8 * (e & 3);
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const float4 x = *reinterpret_cast<const float4*>(re + o + 4 * hf);
        const float4 y = *reinterpret_cast<const float4*>(im + o + 4 * hf);
        float* vr = &v.r[8 * u + 4 * hf];
        float* vi = &v.i[8 * u + 4 * hf];
        vr[0] = x.x; vr[1] = x.y; vr[2] = x.z; vr[3] = x.w;
        vi[0] = y.x; vi[1] = y.y; vi[2] = y.z; vi[3] = y.w;
      }
    }
  }
}

template <bool TALL, bool DIAG>
LRSTV_DEV void bf_stage_fast(const BfChunk& v, __bf16 (*p)[128][kKC + kBfPad], int s) {
  if (TALL) {
    constexpr int NR = DIAG ? 8 : 16;
    const int row = 2 * (s & 63), kb = NR * (s >> 6);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int g = 0; g < NR / 8; ++g) {
        float xr[8], xi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          xr[j] = v.r[2 * (8 * g + j) + c];
          xi[j] = v.i[2 * (8 * g + j) + c];
        }
        bf_split_store(p, row + c, kb + 8 * g, xr, xi);
      }
  } else {
    constexpr int NU = DIAG ? 2 : 4, STEP = DIAG ? 256 : 128;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = s + STEP * u;
      bf_split_store(p, e >> 2, 8 * (e & 3), *reinterpret_cast<const float(*)[8]>(&v.r[8 * u]),
                     *reinterpret_cast<const float(*)[8]>(&v.i[8 * u]));
    }
  }
}

template <bool TALL>
LRSTV_DEV void bf_fetch_slow(BfChunk& v, const float* re, const float* im, int h, int w, int n, int base, int s,
                             int k0) {
  if (TALL) {
    // A(i, k) = conj(M(k, i)), B(k, j) = M(k, j): columns of M, rows k
    const int col = base + 4 * (s & 31), q = s >> 5, nv = col < n ? n - col : 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int k = k0 + 8 * q + r;
      load4(re + (int64_t)k * w + col, k < h ? nv : 0, *reinterpret_cast<float(*)[4]>(&v.r[4 * r]));
      load4(im + (int64_t)k * w + col, k < h ? nv : 0, *reinterpret_cast<float(*)[4]>(&v.i[4 * r]));
    }
  } else {
    // A(i, k) = M(i, k), B(k, j) = conj(M(j, k)): rows of M, k contiguous
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = s + 128 * u, mr = base + (e >> 2), k = k0 + 8 * (e & 3);
      const int nv = (mr < n && k < w) ? w - k : 0;
      load8(re + (int64_t)mr * w + k, nv, *reinterpret_cast<float(*)[8]>(&v.r[8 * u]));
      load8(im + (int64_t)mr * w + k, nv, *reinterpret_cast<float(*)[8]>(&v.i[8 * u]));
    }
  }
}

template <bool TALL>
LRSTV_DEV void bf_stage_slow(const BfChunk& v, __bf16 (*p)[128][kKC + kBfPad], int s) {
  if (TALL) {
    const int c = 4 * (s & 31), q = s >> 5;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      float xr[8], xi[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        xr[r] = v.r[4 * r + cc];
        xi[r] = v.i[4 * r + cc];
      }
      bf_split_store(p, c + cc, 8 * q, xr, xi);
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = s + 128 * u;
      bf_split_store(p, e >> 2, 8 * (e & 3), *reinterpret_cast<const float(*)[8]>(&v.r[8 * u]),
                     *reinterpret_cast<const float(*)[8]>(&v.i[8 * u]));
    }
  }
}

// FAST selects the straight-line staging, DIAG (FAST only) a diagonal tile.
template <bool TALL, bool FAST, bool DIAG>
LRSTV_DEV void bf_fetch(BfChunk& v, const float* re, const float* im, int h, int w, int n, int base, int s, int k0) {
  if (FAST)
    bf_fetch_fast<TALL, DIAG>(v, re, im, h, w, n, base, s, k0);
  else
    bf_fetch_slow<TALL>(v, re, im, h, w, n, base, s, k0);
}
template <bool TALL, bool FAST, bool DIAG>
LRSTV_DEV void bf_stage(const BfChunk& v, __bf16 (*p)[128][kKC + kBfPad], int s) {
  if (FAST)
    bf_stage_fast<TALL, DIAG>(v, p, s);
  else
    bf_stage_slow<TALL>(v, p, s);
}

template <bool TALL, bool FAST, bool DIAG>
LRSTV_DEV void gram_bf16_tile(GramBfSmem& sm, const SliceDesc& d, const float* sl, float2* gram, int ti, int tj) {
  const int n = d.n1, h = d.h, w = d.w, K = TALL ? h : w;
  const float* re = sl + d.a_off;
  const float* im = re + (int64_t)h * w;
  const int i0 = 128 * ti, j0 = 128 * tj;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wy = wv >> 1, wx = wv & 1;
  const int li = lane & 31, lk = lane >> 5;
  f32x16 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) cre[a][b][e] = cim[a][b][e] = 0.f;
  // staging: one panel by all threads on a diagonal tile, else threads
  // 0-127 the row operand (A) and 128-255 the column operand (B)
  const bool isA = DIAG || t < 128;
  const int st = DIAG ? t : t & 127, base = isA ? i0 : j0;
  __bf16(*dstp)[128][kKC + kBfPad] = isA ? sm.a : sm.b;
  __bf16(*bsrc)[128][kKC + kBfPad] = DIAG ? sm.a : sm.b;
  const int nch = (K + kKC - 1) / kKC;
  BfChunk cur, nxt;
  bf_fetch<TALL, FAST, DIAG>(cur, re, im, h, w, n, base, st, 0);
  bf_stage<TALL, FAST, DIAG>(cur, dstp, st);
  bf_fetch<TALL, FAST, DIAG>(cur, re, im, h, w, n, base, st, kKC);
  // no load in flight at the loop entry, so that the waits inside the loop
  // cover only the loads of the previous trip (s_waitcnt vmcnt(0), the
  // other counters at their maxima in the gfx9 encoding)
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  // chunk c's products from registers, while chunk c + 2 is fetched into
  // nxt and chunk c + 1 (held in cur) is split into the buffer (past the
  // end the split is never read)
  for (int c = 0; c < nch; ++c) {
    bf16x8 ar[2][2][4], br[2][2][4];   // [ks][sub-tile][plane]
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ko = 16 * ks + 8 * lk;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ra = 64 * wy + 32 * a + li, rb = 64 * wx + 32 * a + li;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
          ar[ks][a][pl] = *(const bf16x8*)&sm.a[pl][ra][ko];
          br[ks][a][pl] = *(const bf16x8*)&bsrc[pl][rb][ko];
        }
      }
    }
    __syncthreads();   // the buffer is free: every wave holds chunk c in registers
    bf_fetch<TALL, FAST, DIAG>(nxt, re, im, h, w, n, base, st, kKC * (c + 2));
    __builtin_amdgcn_sched_barrier(0);   // the loads issue first
    bf_stage<TALL, FAST, DIAG>(cur, dstp, st);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // The planes hold Re M and Im M as they are, with no conjugation.
      // Tall (A = M^H, B = M): Re G = Re A Re B + Im A' Im B' and
      // Im G = Re A Im B' - Im A' Re B (primes: the stored planes).  Wide
      // (A = M, B = M^H): the same Re G, and Im G the negative of that
      // accumulation, applied at the store.
      bf16x8 na[2][2];   // -Im A' hi, -Im A' lo
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        na[a][0] = bf_neg(ar[ks][a][2]);
        na[a][1] = bf_neg(ar[ks][a][3]);
      }
      // one term at a time over the four sub-tiles; small terms first
#define LRSTV_BF_TERM(ACC, AOP, BPL)                                                       \
  _Pragma("unroll") for (int a = 0; a < 2; ++a) _Pragma("unroll") for (int b = 0; b < 2; ++b) \
      ACC[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AOP, br[ks][b][BPL], ACC[a][b], 0, 0, 0);
      LRSTV_BF_TERM(cre, ar[ks][a][0], 1)
      LRSTV_BF_TERM(cre, ar[ks][a][1], 0)
      LRSTV_BF_TERM(cre, ar[ks][a][2], 3)
      LRSTV_BF_TERM(cre, ar[ks][a][3], 2)
      LRSTV_BF_TERM(cre, ar[ks][a][0], 0)
      LRSTV_BF_TERM(cre, ar[ks][a][2], 2)
      LRSTV_BF_TERM(cim, ar[ks][a][0], 3)
      LRSTV_BF_TERM(cim, ar[ks][a][1], 2)
      LRSTV_BF_TERM(cim, na[a][0], 1)
      LRSTV_BF_TERM(cim, na[a][1], 0)
      LRSTV_BF_TERM(cim, ar[ks][a][0], 2)
      LRSTV_BF_TERM(cim, na[a][0], 0)
#undef LRSTV_BF_TERM
    }
    // interleave: each product followed by three vector ops, an LDS store every sixth
#pragma unroll
    for (int i = 0; i < 96; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
      if (i % 6 == 5) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
    // the copy waits for chunk c + 2's loads: keep it after the products
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
    __syncthreads();   // chunk c + 1 is in the buffer
  }
  // packed lower triangle; the diagonal is real
  float2* g = gram + d.g_off;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = j0 + 64 * wx + 32 * b + li;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = i0 + 64 * wy + 32 * a + 8 * (e >> 2) + 4 * lk + (e & 3);
        if (row < n && col <= row)
          g[packed(row, col)] = make_float2(cre[a][b][e], row == col ? 0.f : TALL ? cim[a][b][e] : -cim[a][b][e]);
      }
    }
}

__global__ void __launch_bounds__(256, 1) k_gram_bf16(const SliceDesc* __restrict__ desc, const float* __restrict__ sl,
                                                      float2* __restrict__ gram, int ntile, int ns,
                                                      const int* __restrict__ halt) {
  __shared__ GramBfSmem sm;
  int tile, slice;
  if (!xcd_tile_slice(ntile, ns, tile, slice)) return;
  const SliceDesc d = desc[slice];
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int T = (d.n1 + 127) / 128;
  int ti = 0, rem = tile;
  while (rem > ti) { rem -= ti + 1; ++ti; }
  if (ti >= T) return;
  const float* re = sl + d.a_off;
  const bool fast = d.w % 4 == 0 && (d.tall ? d.h : d.w) % kKC == 0 && (reinterpret_cast<uintptr_t>(re) & 15) == 0;
  const bool diag = ti == rem;
  if (d.tall) {
    if (fast && diag)
      gram_bf16_tile<true, true, true>(sm, d, sl, gram, ti, rem);
    else if (fast)
      gram_bf16_tile<true, true, false>(sm, d, sl, gram, ti, rem);
    else
      gram_bf16_tile<true, false, false>(sm, d, sl, gram, ti, rem);
  } else {
    if (fast && diag)
      gram_bf16_tile<false, true, true>(sm, d, sl, gram, ti, rem);
    else if (fast)
      gram_bf16_tile<false, true, false>(sm, d, sl, gram, ti, rem);
    else
      gram_bf16_tile<false, false, false>(sm, d, sl, gram, ti, rem);
  }
}

// ---------------------------------------------------------- tridiagonal ---
// Householder reduction of the packed Hermitian Gram, one block per slice.
// Step i: x = A(i+1:, i); H = I - tau v v^H with H x = beta e_1,
// beta = -phase(x_0) ||x||; p = tau A22 v; w = p - (tau/2)(v^H p) v;
// A22 <- A22 - v w^H - w v^H.  Output (doubles, at t_off):
//   [0,n) diag, [n,2n) |beta|, [2n,3n) phase re, [3n,4n) phase im, [4n,5n) tau
// and reflector i stored in column i of the packed triangle (below diag).
template <bool ONCHIP>
__global__ void __launch_bounds__(256) k_tridiag(const SliceDesc* __restrict__ desc, float2* __restrict__ gram,
                                                 double* __restrict__ tri, const int* __restrict__ halt) {
  extern __shared__ float2 sm[];
  __shared__ double red[8];
  __shared__ double s_tau;
  __shared__ float2 s_beta, s_scale;
  const SliceDesc d = desc[blockIdx.x];
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1;
  const int64_t np = (int64_t)n * (n + 1) / 2;
  float2* gA = gram + d.g_off;
  float2* A = ONCHIP ? sm : gA;
  float2* v = ONCHIP ? sm + np : sm;
  float2* p = v + n;
  float2* colacc = p + n;            // [nwaves][n]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* dg = tri + d.t_off;
  double* eab = dg + n;
  double* phr = eab + n;
  double* phi = phr + n;
  double* taus = phi + n;
  if (ONCHIP) {
    for (int64_t e = threadIdx.x; e < np; e += blockDim.x) A[e] = gA[e];
    __syncthreads();
  }
  // exact power-of-two scaling to ||G||_F ~ 1 (see k_tridiag_reg) and deflation
  double fro = 0.0;
  for (int64_t e = threadIdx.x; e < np; e += blockDim.x) {
    const float2 g = A[e];
    fro += ((double)g.x * g.x + (double)g.y * g.y) * 2.0;
  }
  fro = block_sum(fro, red);
  const int ex = fro > 0.0 ? ilogb(sqrt(fro)) : 0;
  const float gsc = ldexpf(1.0f, -ex);
  const double unsc = ldexp(1.0, ex);
  for (int64_t e = threadIdx.x; e < np; e += blockDim.x) A[e] = cscale(A[e], gsc);
  __syncthreads();
  double ph_r = 1.0, ph_i = 0.0;  // running phase (thread 0)
  if (threadIdx.x == 0) { phr[0] = 1.0; phi[0] = 0.0; }
  for (int i = 0; i < n - 1; ++i) {
    const int m = n - 1 - i;
    double nx2 = 0.0;
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      const float2 x = A[packed(i + 1 + r, i)];
      v[r] = x;
      nx2 += (double)x.x * x.x + (double)x.y * x.y;
    }
    nx2 = block_sum(nx2, red);
    if (threadIdx.x == 0) {
      dg[i] = (double)A[packed(i, i)].x * unsc;
      float2 x0 = v[0];
      const double ax02 = (double)x0.x * x0.x + (double)x0.y * x0.y;
      double tau = 0.0;
      if (nx2 <= kDeflate2) x0 = make_float2(0.f, 0.f);
      float2 beta = x0;
      float2 scl = make_float2(0.f, 0.f);
      if (nx2 > kDeflate2 && nx2 - ax02 > 1e-14 * nx2) {
        // v = x - beta e_1 with v_0 = phase (|x_0| + ||x||); normalised to v_0 = 1,
        // which keeps tau = 1 + |x_0| / ||x|| in [1, 2] whatever the column scale.
        const double nx = sqrt(nx2), ax0 = sqrt(ax02);
        const double pr = ax0 > 0.0 ? x0.x / ax0 : 1.0, pi = ax0 > 0.0 ? x0.y / ax0 : 0.0;
        beta = make_float2((float)(-pr * nx), (float)(-pi * nx));
        const double inv = 1.0 / (ax0 + nx);                 // 1 / v_0 = conj(phase) / (|x_0| + ||x||)
        scl = make_float2((float)(pr * inv), (float)(-pi * inv));
        v[0] = make_float2(1.f, 0.f);
        tau = 1.0 + ax0 / nx;
      }
      s_scale = scl;
      s_tau = tau;
      s_beta = beta;
      taus[i] = tau;
      const double br = beta.x, bi = beta.y, ab = sqrt(br * br + bi * bi);
      eab[i] = ab * unsc;
      if (ab > 0.0) {  // ph_{i+1} = ph_i beta / |beta|
        const double ur = br / ab, ui = bi / ab;
        const double nr = ph_r * ur - ph_i * ui, ni = ph_r * ui + ph_i * ur;
        ph_r = nr;
        ph_i = ni;
      }
      phr[i + 1] = ph_r;
      phi[i + 1] = ph_i;
    }
    __syncthreads();
    const float tau = (float)s_tau;
    if (tau != 0.f) {
      const float2 scl = s_scale;
      for (int r = 1 + threadIdx.x; r < m; r += blockDim.x) v[r] = cmul(v[r], scl);
      __syncthreads();
      // p = tau A22 v: wave per row; row part reduced in-wave, column part in registers.
      float2 cacc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) cacc[u] = make_float2(0.f, 0.f);
      for (int rr = wv; rr < m; rr += nw) {
        const float2* row = A + packed(i + 1 + rr, i + 1);
        const float2 vr = v[rr];
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = lane + 64 * u;
          if (c <= rr) {
            const float2 a = row[c];
            acc = cadd(acc, cmul(a, v[c]));
            if (c < rr) cacc[u] = cadd(cacc[u], cmulc(a, vr));
          }
        }
        acc.x = warp_sumf(acc.x);
        acc.y = warp_sumf(acc.y);
        if (lane == 0) p[rr] = acc;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = lane + 64 * u;
        if (c < m) colacc[wv * n + c] = cacc[u];
      }
      __syncthreads();
      double kv = 0.0;
      for (int r = threadIdx.x; r < m; r += blockDim.x) {
        float2 s = p[r];
        for (int q = 0; q < nw; ++q) s = cadd(s, colacc[q * n + r]);
        s = cscale(s, tau);
        p[r] = s;
        const float2 vr = v[r];
        kv += (double)vr.x * s.x + (double)vr.y * s.y;  // Re(conj(v) p)
      }
      kv = block_sum(kv, red);
      const float K = (float)(0.5 * (double)tau * kv);
      for (int r = threadIdx.x; r < m; r += blockDim.x) p[r] = csub(p[r], cscale(v[r], K));
      __syncthreads();
      // A22 <- A22 - v w^H - w v^H (lower part)
      for (int rr = wv; rr < m; rr += nw) {
        float2* row = A + packed(i + 1 + rr, i + 1);
        const float2 vr = v[rr], wr = p[rr];
        for (int c = lane; c <= rr; c += 64) {
          const float2 vc = v[c], wc = p[c];
          // v_r conj(w_c) + w_r conj(v_c)
          const float2 t1 = make_float2(vr.x * wc.x + vr.y * wc.y, vr.y * wc.x - vr.x * wc.y);
          const float2 t2 = make_float2(wr.x * vc.x + wr.y * vc.y, wr.y * vc.x - wr.x * vc.y);
          row[c] = csub(row[c], cadd(t1, t2));
        }
      }
    }
    // store the reflector in column i (below the diagonal)
    for (int r = threadIdx.x; r < m; r += blockDim.x) A[packed(i + 1 + r, i)] = (tau != 0.f) ? v[r] : make_float2(0.f, 0.f);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dg[n - 1] = (double)A[packed(n - 1, n - 1)].x * unsc;
    eab[n - 1] = 0.0;
    taus[n - 1] = 0.0;
  }
  if (ONCHIP) {
    __syncthreads();
    for (int64_t e = threadIdx.x; e < np; e += blockDim.x) gA[e] = A[e];
  }
}

// Householder reduction with the packed Gram held on-chip, for n1 <= 256.
// NW waves.  Rows [RL, n) of the packed lower triangle live in VGPRs:
// row r = RL + wave + NW j (j < JR), lane l holds columns l + 64 u (u < 4);
// rows [0, RL) live in LDS.  RL = max(0, n - NW JR).
// Three barriers per step: (1) after the symmetric product, whose pass also
// accumulates v^H A v, (2) after p and w = p - K v are formed, (3) after the
// rank-2 update, whose pass also extracts the next column, its norm and the
// next diagonal.  Every thread forms the reflector itself from the reduced
// norm; v = [1; scl * x] is applied on the fly from the unscaled column x.
template <int JR, int NW>
__global__ void __launch_bounds__(64 * NW) k_tridiag_reg(const SliceDesc* __restrict__ desc,
                                                         float2* __restrict__ gram, double* __restrict__ tri, const int* __restrict__ halt) {
  extern __shared__ float2 sm[];
  // red_nx and s_dii are written for step i+1 while step i may still read them
  // (the no-reflection path has no barrier in between): double-buffered by parity.
  __shared__ double red_nx[2][NW], red_vav[NW];
  __shared__ double s_dii[2];
  const SliceDesc d = desc[blockIdx.x];
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1;
  const int RL = n > NW * JR ? n - NW * JR : 0;
  const int64_t npl = (int64_t)RL * (RL + 1) / 2;
  float2* gA = gram + d.g_off;
  float2* A = sm;                    // rows [0, RL), packed
  float2* xb0 = sm + npl;            // [n] column below the diagonal (double-buffered)
  float2* xb1 = xb0 + n;             // [n]
  float2* wb = xb1 + n;              // [n] row parts of A v, then w
  float2* colacc = wb + n;           // [NW][n]
  const int lane = threadIdx.x & 63;
  // wave index as a wave-uniform (scalar) value, so that row and slot tests
  // below become scalar branches instead of per-lane predication
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* dg = tri + d.t_off;
  double* eab = dg + n;
  double* phr = eab + n;
  double* phi = phr + n;
  double* taus = phi + n;
  float2 reg[JR][4];
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    const int r = RL + wv + NW * j;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = lane + 64 * u;
      reg[j][u] = (r < n && c <= r) ? gA[packed(r, c)] : make_float2(0.f, 0.f);
    }
  }
  for (int64_t e = threadIdx.x; e < npl; e += blockDim.x) A[e] = gA[e];
  // Scale by an exact power of two so that ||G||_F ~ 1: no FP32 denormals or
  // overflow in the reflectors whatever the slice's magnitude.  Columns whose
  // norm falls below kDeflate (relative to ||G||_F, under the FP32 Gram's own
  // resolution) are rounding residue and are deflated (beta = 0, a split).
  double fro = 0.0;
  for (int64_t e = threadIdx.x; e < npl; e += blockDim.x) {
    const float2 g = A[e];
    fro += ((double)g.x * g.x + (double)g.y * g.y) * 2.0;
  }
#pragma unroll
  for (int j = 0; j < JR; ++j)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float2 g = reg[j][u];
      fro += ((double)g.x * g.x + (double)g.y * g.y) * 2.0;
    }
  fro = warp_sum(fro);
  if (lane == 0) red_vav[wv] = fro;
  __syncthreads();
  double fro2 = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) fro2 += red_vav[q];
  const int ex = fro2 > 0.0 ? ilogb(sqrt(fro2)) : 0;
  const float gsc = ldexpf(1.0f, -ex);
  const double unsc = ldexp(1.0, ex);
  for (int64_t e = threadIdx.x; e < npl; e += blockDim.x) A[e] = cscale(A[e], gsc);
#pragma unroll
  for (int j = 0; j < JR; ++j)
#pragma unroll
    for (int u = 0; u < 4; ++u) reg[j][u] = cscale(reg[j][u], gsc);
  __syncthreads();
  // column 0, its norm and the diagonal A(0, 0)
  {
    double part = 0.0;
    for (int r = 1 + threadIdx.x; r < n; r += blockDim.x) {
      float2 x;
      if (r < RL) x = A[packed(r, 0)];
      else x = make_float2(0.f, 0.f);
      if (r < RL) {
        xb0[r - 1] = x;
        part += (double)x.x * x.x + (double)x.y * x.y;
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < JR; ++j) {
        const int r = RL + wv + NW * j;
        if (r >= 1 && r < n) {
          const float2 x = reg[j][0];
          xb0[r - 1] = x;
          part += (double)x.x * x.x + (double)x.y * x.y;
        }
        if (r == 0) s_dii[0] = (double)reg[j][0].x;
      }
    }
    if (threadIdx.x == 0 && RL > 0) s_dii[0] = (double)A[0].x;
    part = warp_sum(part);
    if (lane == 0) red_nx[0][wv] = part;
  }
  __syncthreads();
  double ph_r = 1.0, ph_i = 0.0;
  if (threadIdx.x == 0) { phr[0] = 1.0; phi[0] = 0.0; }
  for (int i = 0; i < n - 1; ++i) {
    const int m = n - 1 - i;
    float2* x = (i & 1) ? xb1 : xb0;
    float2* xn = (i & 1) ? xb0 : xb1;
    const int cur = i & 1, nxt = cur ^ 1;
    double nx2 = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) nx2 += red_nx[cur][q];
    const double dii = s_dii[cur];
    // reflector: H x = beta e_1, v = [1; scl x_{1:}], tau in [1, 2]
    float2 x0 = x[0];
    const double ax02 = (double)x0.x * x0.x + (double)x0.y * x0.y;
    double taud = 0.0;
    if (nx2 <= kDeflate2) x0 = make_float2(0.f, 0.f);
    float2 beta = x0, scl = make_float2(0.f, 0.f);
    if (nx2 > kDeflate2 && nx2 - ax02 > 1e-14 * nx2) {
      const double nx = sqrt(nx2), ax0 = sqrt(ax02);
      const double pr = ax0 > 0.0 ? x0.x / ax0 : 1.0, pi = ax0 > 0.0 ? x0.y / ax0 : 0.0;
      beta = make_float2((float)(-pr * nx), (float)(-pi * nx));
      const double inv = 1.0 / (ax0 + nx);
      scl = make_float2((float)(pr * inv), (float)(-pi * inv));
      taud = 1.0 + ax0 / nx;
    }
    if (threadIdx.x == 0) {
      dg[i] = dii * unsc;
      taus[i] = taud;
      const double br = beta.x, bi = beta.y, ab = sqrt(br * br + bi * bi);
      eab[i] = ab * unsc;
      if (ab > 0.0) {
        const double ur = br / ab, uq = bi / ab;
        const double nr = ph_r * ur - ph_i * uq, ni = ph_r * uq + ph_i * ur;
        ph_r = nr;
        ph_i = ni;
      }
      phr[i + 1] = ph_r;
      phi[i + 1] = ph_i;
    }
    const float tau = (float)taud;
    auto vget = [&](int k) -> float2 { return k == 0 ? make_float2(1.f, 0.f) : cmul(scl, x[k]); };
    // per-lane copies of v at this lane's columns (absolute column c = lane + 64 u)
    float2 vc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = lane + 64 * u;
      vc[u] = make_float2(0.f, 0.f);
      if (64 * u + 63 > i && 64 * u < n && c > i && c < n) vc[u] = vget(c - i - 1);
    }
    double nxp = 0.0;
    const float2 zero = make_float2(0.f, 0.f);
    if (tau != 0.f) {
      // (1) row parts of A v (in-wave reduce), column parts by absolute column, v^H A v
      float2 cacc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cacc[u] = zero;
      double vav = 0.0;
      for (int r = i + 1 + wv; r < RL; r += NW) {
        const float2* row = A + packed(r, 0);
        const float2 vr = vget(r - i - 1);
        float2 acc = zero;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (64 * u + 63 <= i || 64 * u > r) continue;   // uniform: slot outside (i, r]
          const int c = lane + 64 * u;
          if (c > i && c <= r) {
            const float2 a = row[c];
            acc = cadd(acc, cmul(a, vc[u]));
            if (c < r) cacc[u] = cadd(cacc[u], cmulc(a, vr));
            else vav -= ((double)vr.x * vr.x + (double)vr.y * vr.y) * a.x;
          }
        }
        acc.x = wave_sumf_dpp(acc.x);
        acc.y = wave_sumf_dpp(acc.y);
        if (lane == 0) {
          wb[r - i - 1] = acc;
          vav += 2.0 * ((double)vr.x * acc.x + (double)vr.y * acc.y);
        }
      }
#pragma unroll
      for (int j = 0; j < JR; ++j) {
        const int r = RL + wv + NW * j;
        if (r > i && r < n) {
          const float2 vr = vget(r - i - 1);
          float2 acc = zero;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (64 * u + 63 <= i || 64 * u > r) continue;
            const int c = lane + 64 * u;
            if (c > i && c <= r) {
              const float2 a = reg[j][u];
              acc = cadd(acc, cmul(a, vc[u]));
              if (c < r) cacc[u] = cadd(cacc[u], cmulc(a, vr));
              else vav -= ((double)vr.x * vr.x + (double)vr.y * vr.y) * a.x;
            }
          }
          acc.x = wave_sumf_dpp(acc.x);
          acc.y = wave_sumf_dpp(acc.y);
          if (lane == 0) {
            wb[r - i - 1] = acc;
            vav += 2.0 * ((double)vr.x * acc.x + (double)vr.y * acc.y);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (64 * u + 63 <= i || 64 * u >= n) continue;
        const int c = lane + 64 * u;
        if (c > i && c < n) colacc[wv * n + c] = cacc[u];
      }
      vav = warp_sum(vav);
      if (lane == 0) red_vav[wv] = vav;
      __syncthreads();
      // (2) p = tau A v, K = tau^2 v^H A v / 2, w = p - K v
      double vAv = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) vAv += red_vav[q];
      const float K = (float)(0.5 * taud * taud * vAv);
      for (int rr = threadIdx.x; rr < m; rr += blockDim.x) {
        const int c = i + 1 + rr;
        float2 sacc = wb[rr];
#pragma unroll
        for (int q = 0; q < NW; ++q) sacc = cadd(sacc, colacc[q * n + c]);
        wb[rr] = csub(cscale(sacc, tau), cscale(vget(rr), K));
      }
      __syncthreads();
      // (3) A22 <- A22 - v w^H - w v^H; column i <- v; next column -> xn
      float2 wc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = lane + 64 * u;
        wc[u] = zero;
        if (64 * u + 63 > i && 64 * u < n && c > i && c < n) wc[u] = wb[c - i - 1];
      }
      for (int r = i + 1 + wv; r < RL; r += NW) {
        float2* row = A + packed(r, 0);
        const float2 vr = vget(r - i - 1), wr = wb[r - i - 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (64 * u + 63 <= i || 64 * u > r) continue;
          const int c = lane + 64 * u;
          if (c > i && c <= r) {
            const float2 t1 = make_float2(vr.x * wc[u].x + vr.y * wc[u].y, vr.y * wc[u].x - vr.x * wc[u].y);
            const float2 t2 = make_float2(wr.x * vc[u].x + wr.y * vc[u].y, wr.y * vc[u].x - wr.x * vc[u].y);
            const float2 a = csub(row[c], cadd(t1, t2));
            row[c] = a;
            if (c == i + 1) {
              if (r > i + 1) {
                xn[r - i - 2] = a;
                nxp += (double)a.x * a.x + (double)a.y * a.y;
              } else {
                s_dii[nxt] = (double)a.x;
              }
            }
          }
        }
        if (lane == (i & 63)) row[i] = vr;   // reflector column (c = i lives in slot i >> 6)
      }
#pragma unroll
      for (int j = 0; j < JR; ++j) {
        const int r = RL + wv + NW * j;
        if (r > i && r < n) {
          const float2 vr = vget(r - i - 1), wr = wb[r - i - 1];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (64 * u + 63 < i || 64 * u > r) continue;   // slot holds neither column i nor (i, r]
            const int c = lane + 64 * u;
            if (c > i && c <= r) {
              const float2 t1 = make_float2(vr.x * wc[u].x + vr.y * wc[u].y, vr.y * wc[u].x - vr.x * wc[u].y);
              const float2 t2 = make_float2(wr.x * vc[u].x + wr.y * vc[u].y, wr.y * vc[u].x - wr.x * vc[u].y);
              const float2 a = csub(reg[j][u], cadd(t1, t2));
              reg[j][u] = a;
              if (c == i + 1) {
                if (r > i + 1) {
                  xn[r - i - 2] = a;
                  nxp += (double)a.x * a.x + (double)a.y * a.y;
                } else {
                  s_dii[nxt] = (double)a.x;
                }
              }
            }
            if (c == i) reg[j][u] = vr;    // reflector column
          }
        }
      }
    } else {
      // no reflection: column i stores zeros; extract the next column unchanged
      for (int r = i + 1 + wv; r < RL; r += NW) {
        float2* row = A + packed(r, 0);
        if (lane == (i & 63)) row[i] = zero;
        if (lane == ((i + 1) & 63)) {
          const float2 a = row[i + 1];
          if (r > i + 1) {
            xn[r - i - 2] = a;
            nxp += (double)a.x * a.x + (double)a.y * a.y;
          } else {
            s_dii[nxt] = (double)a.x;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < JR; ++j) {
        const int r = RL + wv + NW * j;
        if (r > i && r < n) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int c = lane + 64 * u;
            if (c == i) reg[j][u] = zero;
            if (c == i + 1) {
              const float2 a = reg[j][u];
              if (r > i + 1) {
                xn[r - i - 2] = a;
                nxp += (double)a.x * a.x + (double)a.y * a.y;
              } else {
                s_dii[nxt] = (double)a.x;
              }
            }
          }
        }
      }
    }
    nxp = warp_sum(nxp);
    if (lane == 0) red_nx[nxt][wv] = nxp;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dg[n - 1] = s_dii[(n - 1) & 1] * unsc;
    eab[n - 1] = 0.0;
    taus[n - 1] = 0.0;
  }
  // write back: only the reflectors (strict lower part) are used afterwards
  for (int64_t e = threadIdx.x; e < npl; e += blockDim.x) gA[e] = A[e];
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    const int r = RL + wv + NW * j;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = lane + 64 * u;
      if (r < n && c <= r) gA[packed(r, c)] = reg[j][u];
    }
  }
}

// ------------------------------------ tridiagonalisation on MFMA tiles ---
// The same Householder reduction (same reflector convention and outputs as
// k_tridiag_reg) with the whole Hermitian Gram held in registers as 32 x 32
// tiles in the matrix-core accumulator layout: lane l, element r of tile
// (R, C) is G(32 R + rho(r, l / 32), 32 C + l % 32), rho(r, h) =
// 8 (r / 4) + 4 h + r % 4.  Lower tiles (R >= C) only; the diagonal tiles
// hold both triangles.  NW waves hold TPW tiles each, dealt column-major.
//
// The product is formed with the raw column x (column i below the
// diagonal) instead of the reflector v = scl x + gamma e_{i+1} (gamma =
// 1 - scl x_{i+1}, real, in [1/2, 1]):
//   A v = scl (A x) + gamma a,   a = column i+1 of the trailing matrix,
//   v^H A v = |scl|^2 x^H A x + 2 gamma Re(conj(scl) x^H a) + gamma^2 a_{i+1},
// and the next step's columns are formed from this step's, without waiting
// for the update on the matrix cores: column c of the updated matrix is
// a_c - v conj(w_c) - w conj(v_c).  Two barriers per step i:
//   C  per tile the column sums conj(a) x_row are lane-local (halves
//      combined) and give the whole product of a diagonal tile; the row sums
//      a x_col of an off-diagonal tile are reduced across the lanes in
//      registers (lane exchanges, no LDS traffic).  Partial sums per wave,
//      x^H A x partials; column i+2 out of the tiles
//   D  one index per thread of the first four waves: v, w = tau A v -
//      (tau^2 v^H A v / 2) v, the reflector column to the Gram; the next x
//      (column i+1 of the updated matrix), a (column i+2), diagonal, ||x||^2
//      and x^H a partials
//   E  A -= v w^H + w v^H on the matrix cores (per tile four
//      v_mfma_f32_32x32x2f32: real and imaginary parts as rank-4 real
//      products); meanwhile every thread forms the next reflector.
LRSTV_DEV int mt_rho(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// x of lane l plus x of lane l ^ 32, in every lane (the two halves swapped
// across the wave by v_permlane32_swap)
LRSTV_DEV float half_pair_sum(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Lanes 0-15 of each 32-lane half: x + x of lane l + 16; lanes 16-31: y + y
// of lane l - 16 (v_permlane16_swap exchanges lanes 16-31 of x with lanes
// 0-15 of y).
LRSTV_DEV float lane_pair16_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// One halving step of a register reduction: of v[0 .. 2M), the lane keeps
// v[m + M sel] and adds the partner's copy of it (the partner, given by the
// DPP control CTRL, has the other sel and sends v[m + M (1 - sel)] in turn).
template <int M, int CTRL>
LRSTV_DEV void row_halve(float* v, int sel) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const float keep = sel ? v[m + M] : v[m], send = sel ? v[m] : v[m + M];
    v[m] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xf, 0xf, false));
  }
}


// tile t of the column-major enumeration of the lower tiles of an NT x NT grid
LRSTV_DEV void mt_tile(int t, int NT, int& R, int& C) {
  C = 0;
  while (t >= NT - C) {
    t -= NT - C;
    ++C;
  }
  R = C + t;
}

// Column c of the register tiles (all rows of the tiles holding it) into
// dst; with below, rows <= c within its block are written as zeros and the
// diagonal goes to *dii.  The element rows are compared through rel, which
// changes with c, so that no per-element row index stays live across the
// step loop.
template <int TPW>
LRSTV_DEV void mt_column(const f32x16 (&tre)[TPW], const f32x16 (&tim)[TPW], const int (&tR)[TPW],
                         const int (&tC)[TPW], int c, int li, int h, float2* dst, bool below, double* dii) {
  const int cb = c >> 5, cl = c & 31;
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    if (tC[s] != cb) continue;   // uniform
    if (li == cl) {
      const int rel = c - 32 * tR[s] - 4 * h;
      float2* d = dst + 32 * tR[s] + 4 * h;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int cr = mt_rho(r, 0);
        float2 a = make_float2(tre[s][r], tim[s][r]);
        if (below && cr <= rel) {
          if (cr == rel) *dii = (double)a.x;
          a = make_float2(0.f, 0.f);
        }
        d[cr] = a;
      }
    }
  }
}

// Reflector H x = beta e_1, v = [1; scl x], tau in [1, 2], from ||x||^2, x_0
// (equal in every lane: kept in scalar registers).  The deflation tests in
// FP64, the factors in FP32, the precision of the tiles they apply to.
struct MtRefl {
  float ax0, pr, pim, nx, tau, gam;
  float2 scl;
  bool refl, defl;
};
LRSTV_DEV MtRefl mt_reflector(double nx2, float2 x0) {
  MtRefl f;
  const double ax02 = (double)x0.x * x0.x + (double)x0.y * x0.y;
  f.defl = nx2 <= kDeflate2;
  f.refl = !f.defl && nx2 - ax02 > 1e-14 * nx2;
  // hardware square root and reciprocal (about 1 ulp): FP32 factors of an
  // FP32 reduction
  f.ax0 = uniform_f(__builtin_amdgcn_sqrtf((float)ax02));
  const float rax = f.ax0 > 0.f ? __builtin_amdgcn_rcpf(f.ax0) : 0.f;
  f.pr = uniform_f(f.ax0 > 0.f ? x0.x * rax : 1.f);
  f.pim = uniform_f(f.ax0 > 0.f ? x0.y * rax : 0.f);
  f.nx = 0.f;
  f.tau = 0.f;
  f.gam = 0.f;
  f.scl = make_float2(0.f, 0.f);
  if (f.refl) {
    f.nx = uniform_f(__builtin_amdgcn_sqrtf((float)nx2));
    const float inv = __builtin_amdgcn_rcpf(f.ax0 + f.nx);
    f.scl = make_float2(uniform_f(f.pr * inv), uniform_f(-f.pim * inv));
    f.tau = uniform_f(1.f + f.ax0 * __builtin_amdgcn_rcpf(f.nx));
    f.gam = uniform_f(f.nx * inv);
  }
  return f;
}

// NMAX: the largest n of the shape (256, or 128 for a 4-wave block of
// which three fit a CU); the launch takes the slices with nmin < n <= NMAX.
template <int NW, int TPW, int NMAX = 256>
__global__ void __launch_bounds__(64 * NW, NMAX == 256 ? 1 : 3) k_tridiag_mfma(const SliceDesc* __restrict__ desc,
                                                         float2* __restrict__ gram, double* __restrict__ tri,
                                                         const int* __restrict__ halt, int nmin) {
  constexpr int NDW = NMAX / 64;   // waves of D, one index per thread
  constexpr int NTM = NMAX / 32;
  static_assert(NMAX % 64 == 0 && NW * TPW >= NTM * (NTM + 1) / 2, "the lower 32 x 32 tiles of an NMAX x NMAX Gram");
  static_assert(NW >= NDW, "one index per thread in D");
  // columns i, i+1 (by step parity) and i+2 of the current matrix
  __shared__ float2 xb[2][NMAX], ab[2][NMAX], bb[NMAX];
  __shared__ float2 vb[NMAX], wb[NMAX];
  __shared__ float2 P[NW][NMAX];               // per-wave partial sums of A x
  // per-wave partial sums (FP32 within a wave, summed over the waves in FP64)
  __shared__ float red_nx[2][NW], red_xa[2][NW][2], red_xax[NW];
  __shared__ double red_fro[NW];
  __shared__ double s_dii[2];
  const SliceDesc d = desc[blockIdx.x];
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1;
  if (n <= nmin || n > NMAX) return;   // another launch takes it (nmin >= 0)
  const int NT = (n + 31) >> 5, ntile = NT * (NT + 1) / 2;
  float2* gA = gram + d.g_off;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* dg = tri + d.t_off;
  double* eab = dg + n;
  double* phr = eab + n;
  double* phi = phr + n;
  double* taus = phi + n;
  const float2 zero = make_float2(0.f, 0.f);
  // ---- load the tiles ----------------------------------------------------
  f32x16 tre[TPW], tim[TPW];
  int tR[TPW], tC[TPW];
  {
    const int lane = threadIdx.x & 63, li = lane & 31, h = lane >> 5;
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      const int t = wv + NW * s;
      int R = -1, C = -1;
      if (t < ntile) mt_tile(t, NT, R, C);
      tR[s] = R;
      tC[s] = C;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float2 a = zero;
        if (R >= 0) {
          const int row = 32 * R + mt_rho(r, h), col = 32 * C + li;
          if (row < n && col < n) a = row >= col ? gA[packed(row, col)] : cconj(gA[packed(col, row)]);
        }
        tre[s][r] = a.x;
        tim[s][r] = a.y;
      }
    }
  }
  // ---- exact power-of-two scaling to ||G||_F ~ 1 (as in k_tridiag_reg) ----
  double fro = 0.0;
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const double wgt = tR[s] == tC[s] ? 1.0 : 2.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) fro += wgt * ((double)tre[s][r] * tre[s][r] + (double)tim[s][r] * tim[s][r]);
  }
  fro = wave_sum_dpp(fro);
  if ((threadIdx.x & 63) == 0) red_fro[wv] = fro;
  __syncthreads();
  double fro2 = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) fro2 += red_fro[q];
  const int ex = fro2 > 0.0 ? ilogb(sqrt(fro2)) : 0;
  const float gsc = ldexpf(1.0f, -ex);
  const double unsc = uniform_d(ldexp(1.0, ex));
#pragma unroll
  for (int s = 0; s < TPW; ++s)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      tre[s][r] *= gsc;
      tim[s][r] *= gsc;
    }
  double ph_r = 1.0, ph_i = 0.0;   // running phase (uniform in the waves of D)
  if (threadIdx.x == 0) { phr[0] = 1.0; phi[0] = 0.0; }
  // columns 0 and 1; ||x||^2 and x^H a of step 0; its reflector
  {
    const int lane = threadIdx.x & 63, li = lane & 31, h = lane >> 5;
    mt_column<TPW>(tre, tim, tR, tC, 0, li, h, xb[0], true, &s_dii[0]);
    mt_column<TPW>(tre, tim, tR, tC, 1, li, h, ab[0], false, nullptr);
  }
  __syncthreads();
  {
    const int t = threadIdx.x;
    float nn = 0.f, xr = 0.f, xi = 0.f;
    if (t < NMAX && t > 0 && t < n) {
      const float2 x = xb[0][t], a1 = ab[0][t];
      nn = x.x * x.x + x.y * x.y;
      const float2 p = cmulc(x, a1);
      xr = p.x;
      xi = p.y;
    }
    nn = wave_sumf_dpp(nn);
    xr = wave_sumf_dpp(xr);
    xi = wave_sumf_dpp(xi);
    if ((threadIdx.x & 63) == 0) {
      red_nx[0][wv] = nn;
      red_xa[0][wv][0] = xr;
      red_xa[0][wv][1] = xi;
    }
  }
  __syncthreads();
  // The reflector of a step is needed by the waves of D only: without a
  // reflection D writes v = w = 0, so that C's products are discarded and E
  // adds zeros.  That of step i + 1 is formed right after the barrier that
  // ends D of step i by one wave outside D that has slack in C (WR: with 12
  // waves, wave 9, whose tiles include two diagonal ones) and passed to D
  // through LDS, so that it is off the path of the waves of D (D, then
  // their share of E and C); with every wave in D (4-wave shape) the waves
  // of D form it themselves.
  constexpr int WR = NW == 12 ? 9 : (NW > NDW ? NW - 1 : -1);
  __shared__ MtRefl s_f;
  MtRefl f{};
  auto next_reflector = [&](int pr, int i1) {
    double nx2 = 0.0;
#pragma unroll
    for (int q = 0; q < NDW; ++q) nx2 += red_nx[pr][q];
    return mt_reflector(uniform_d(nx2), make_float2(uniform_f(xb[pr][i1].x), uniform_f(xb[pr][i1].y)));
  };
  auto form_reflector = [&](int pr, int i1) {
    if (WR < 0) {
      if (wv < NDW) f = next_reflector(pr, i1);
    } else if (wv == WR) {
      const MtRefl g = next_reflector(pr, i1);
      if ((threadIdx.x & 63) == 0) s_f = g;
    }
  };
  if (n > 1) form_reflector(0, 1);
  // Issue priority by share of tiles: the waves holding the most tiles set
  // the length of the product and update phases, the waves of D have slack
  // there (the tile dealing gives waves 8-11 the most).
  if (wv >= 8) __builtin_amdgcn_s_setprio(2);
  else if (wv >= NDW) __builtin_amdgcn_s_setprio(1);
  for (int i = 0; i < n - 1; ++i) {
    const int par = i & 1;
    const float2* xv = xb[par];
    const float2* av = ab[par];
    // lane-derived indices are recomputed every step from this copy rather
    // than kept live across the loop next to the tiles
    const int lane = opaque_i(threadIdx.x & 63), li = lane & 31, h = lane >> 5;
    // ---- C: A x per wave, x^H A x ----------------------------------------
    {
      for (int t = lane; t < NMAX; t += 64) P[wv][t] = zero;
      float xaxd = 0.f, xaxo = 0.f;   // diagonal-tile and off-diagonal-tile parts
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        const int R = tR[s], C = tC[s];
        if (R < 0 || 32 * C + 31 <= i) continue;   // no element in the trailing block
        const int col = 32 * C + li;
        // the partial sums this tile adds to, read first so that their
        // latency is covered by the products
        float* Pf = reinterpret_cast<float*>(P[wv]);
        const int rsel = 2 * (32 * R + mt_rho(li >> 1, h)) + (li & 1);   // see the row sums below
        const float2 pcol = P[wv][col];
        const float prow = R != C ? Pf[rsel] : 0.f;
        const float2 xC = xv[col];
        // column sums conj(a) x_row as four FMAs per element
        float cr = 0.f, ci = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float ar = tre[s][r], ai = tim[s][r];
          const float2 xr = xv[32 * R + mt_rho(r, h)];
          cr = fmaf(ar, xr.x, cr);
          cr = fmaf(ai, xr.y, cr);
          ci = fmaf(ar, xr.y, ci);
          ci = fmaf(-ai, xr.x, ci);
        }
        // Re(conj(x_col) (A^H x)_col); twice for an off-diagonal tile (its mirror)
        if (R == C) xaxd += cr * xC.x + ci * xC.y;
        else xaxo += cr * xC.x + ci * xC.y;
        // both halves of the column (lanes l and l + 32) summed in every lane
        const float2 csum = make_float2(half_pair_sum(cr), half_pair_sum(ci));
        if (h == 0) P[wv][col] = cadd(pcol, csum);
        if (R != C) {
          // row sums of a x_col over the 32 lanes of each half, in registers:
          // value k = 2 r + c (c: real / imaginary part of row rho(r, h)) is
          // halved five times, lane bit 4, 3, 2, 1, 0 choosing the half it
          // keeps while the partner (lane ^ 16, ^ 15, ^ 7, ^ 3, ^ 1) adds the
          // other, so that lane li ends with the sum of value k = li
          float v[32];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float2 pr = cmul(make_float2(tre[s][r], tim[s][r]), xC);
            v[2 * r] = pr.x;
            v[2 * r + 1] = pr.y;
          }
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j] = lane_pair16_sum(v[j], v[j + 16]);
          row_halve<8, 0x140>(v, (li >> 3) & 1);   // partner lane ^ 15 (row mirror)
          row_halve<4, 0x141>(v, (li >> 2) & 1);   // lane ^ 7 (half-row mirror)
          row_halve<2, 0x1B>(v, (li >> 1) & 1);    // lane ^ 3
          row_halve<1, 0xB1>(v, li & 1);           // lane ^ 1
          Pf[rsel] = prow + v[0];
        }
      }
      const float sx = wave_sumf_dpp(xaxd + 2.f * xaxo);
      if (lane == 0) red_xax[wv] = sx;
    }
    // column i+2 of the current matrix
    if (i + 2 < n) mt_column<TPW>(tre, tim, tR, tC, i + 2, li, h, bb, false, nullptr);
    lds_barrier();
    // ---- D: v, w; the reflector column; the next x, a, diagonal ------------
    // Without a reflection v and w are zero (selects, so that stale partial
    // sums do not enter).
    if (wv < NDW) {
      // the reflector formed outside D: read here, made uniform where it is
      // first used (after the partial sums' reads are in flight)
      MtRefl fs{};
      if (WR >= 0) fs = s_f;
      const int t = threadIdx.x;
      const int i1 = i + 1, i2 = i + 2 < n ? i + 2 : i + 1;
      // Values equal for every index (the reduced scalars, the partial sums at
      // i+1 and i+2) are summed across the wave, lane q holding wave q's
      // part, and land in scalar registers.
      double xAx = 0.0, xar = 0.0, xai = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) xAx += red_xax[q];
#pragma unroll
      for (int q = 0; q < NDW; ++q) {
        xar += red_xa[par][q][0];
        xai += red_xa[par][q][1];
      }
      const int ql = lane < NW ? lane : 0;
      const bool qa = lane < NW;
      const float2 p1 = qa ? P[ql][i1] : zero, p2 = qa ? P[ql][i2] : zero;
      const float2 S1 = make_float2(wave_sumf_dpp(p1.x), wave_sumf_dpp(p1.y));
      const float2 S2 = make_float2(wave_sumf_dpp(p2.x), wave_sumf_dpp(p2.y));
      const float2 a1 = make_float2(uniform_f(av[i1].x), uniform_f(av[i1].y));
      const float2 a2 = make_float2(uniform_f(av[i2].x), uniform_f(av[i2].y));
      const float2 x2 = make_float2(uniform_f(xv[i2].x), uniform_f(xv[i2].y));
      float2 St = zero;
#pragma unroll
      for (int q = 0; q < NW; ++q) St = cadd(St, P[q][t]);
      const float2 at = av[t], xt = xv[t], bt = bb[t];
      if (WR >= 0) {
        f.ax0 = uniform_f(fs.ax0);
        f.pr = uniform_f(fs.pr);
        f.pim = uniform_f(fs.pim);
        f.nx = uniform_f(fs.nx);
        f.tau = uniform_f(fs.tau);
        f.gam = uniform_f(fs.gam);
        f.scl = make_float2(uniform_f(fs.scl.x), uniform_f(fs.scl.y));
        f.refl = __builtin_amdgcn_readfirstlane((int)fs.refl) != 0;
        f.defl = __builtin_amdgcn_readfirstlane((int)fs.defl) != 0;
      }
      const double sr = f.scl.x, si = f.scl.y;
      const double gd = f.gam, td = f.tau;
      const double vAv = (sr * sr + si * si) * xAx + 2.0 * gd * (sr * xar + si * xai) + gd * gd * (double)a1.x;
      const float K = (float)(0.5 * td * td * vAv), g = f.gam, tau = f.tau;
      // w_u = tau (scl S_u + gamma a_u) - K v_u
      auto w_of = [&](float2 S, float2 au, float2 vu) {
        const float2 pu = cadd(cmul(f.scl, S), make_float2(g * au.x, g * au.y));
        return make_float2(tau * pu.x - K * vu.x, tau * pu.y - K * vu.y);
      };
      const bool in = f.refl && t > i && t < n;
      const float2 v2 = (f.refl && i + 2 < n) ? cmul(f.scl, x2) : zero;
      const float2 v = !in ? zero : t == i1 ? make_float2(1.f, 0.f) : cmul(f.scl, xt);
      const float2 w1 = f.refl ? w_of(S1, a1, make_float2(1.f, 0.f)) : zero;
      const float2 w2 = (f.refl && i + 2 < n) ? w_of(S2, a2, v2) : zero;
      const float2 w = in ? w_of(St, at, v) : zero;
      // updated columns i+1 and i+2: a_c - v conj(w_c) - w conj(v_c)
      const bool nxt = t > i1 && t < n;
      const float2 xn = !nxt ? zero : make_float2(at.x - (v.x * w1.x + v.y * w1.y) - w.x, at.y - (v.y * w1.x - v.x * w1.y) - w.y);
      const float2 an = !nxt ? zero : make_float2(bt.x - (v.x * w2.x + v.y * w2.y) - (w.x * v2.x + w.y * v2.y),
                                                  bt.y - (v.y * w2.x - v.x * w2.y) - (w.y * v2.x - w.x * v2.y));
      float nn = 0.f, xr = 0.f, xi = 0.f;
      if (nxt) {
        nn = xn.x * xn.x + xn.y * xn.y;
        const float2 pxa = cmulc(xn, an);
        xr = pxa.x;
        xi = pxa.y;
      }
      vb[t] = v;
      wb[t] = w;
      xb[par ^ 1][t] = xn;
      ab[par ^ 1][t] = an;
      if (t == i1) s_dii[par ^ 1] = (double)a1.x - 2.0 * (double)w1.x;
      if (t > i && t < n) gA[packed(t, i)] = v;   // reflector column (zeros without a reflection)
      nn = wave_sumf_dpp(nn);
      xr = wave_sumf_dpp(xr);
      xi = wave_sumf_dpp(xi);
      if (lane == 0) {
        red_nx[par ^ 1][wv] = nn;
        red_xa[par ^ 1][wv][0] = xr;
        red_xa[par ^ 1][wv][1] = xi;
      }
      // outputs of step i; beta = -phase ||x|| (reflection), x_0 (column
      // already reduced) or 0 (deflated); the running phase is uniform
      if (!f.defl) {
        const double ur = f.refl ? -f.pr : f.pr, uq = f.refl ? -f.pim : f.pim;
        const double nr = ph_r * ur - ph_i * uq, ni = ph_r * uq + ph_i * ur;
        ph_r = uniform_d(nr);
        ph_i = uniform_d(ni);
      }
      if (t == 0) {
        dg[i] = s_dii[par] * unsc;
        taus[i] = f.tau;
        eab[i] = (double)(f.refl ? f.nx : f.defl ? 0.f : f.ax0) * unsc;
        phr[i + 1] = ph_r;
        phi[i + 1] = ph_i;
      }
    }
    lds_barrier();
    if (i + 2 < n) form_reflector(par ^ 1, i + 2);
    // ---- E: A -= v w^H + w v^H on the matrix cores ------------------------
    // real part: [-v_R | -w_R] (re in half 0, im in half 1) times [w_C ; v_C];
    // imaginary part: [-Im v, Re v] and [-Im w, Re w] against the same B.
    {
      // every tile's v and w entries are read before the first product, so
      // that one LDS latency covers them all
      float2 vRs[TPW], wRs[TPW], vCs[TPW], wCs[TPW];
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        const int R = tR[s] < 0 ? 0 : tR[s], C = tC[s] < 0 ? 0 : tC[s];
        vRs[s] = vb[32 * R + li];
        wRs[s] = wb[32 * R + li];
        vCs[s] = vb[32 * C + li];
        wCs[s] = wb[32 * C + li];
      }
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        const int R = tR[s], C = tC[s];
        if (R < 0 || 32 * C + 31 <= i) continue;
        const float2 vR = vRs[s], wR = wRs[s], vC = vCs[s], wC = wCs[s];
        const float b0 = h ? wC.y : wC.x, b1 = h ? vC.y : vC.x;
        const float ar0 = h ? -vR.y : -vR.x, ar1 = h ? -wR.y : -wR.x;
        const float ai0 = h ? vR.x : -vR.y, ai1 = h ? wR.x : -wR.y;
        tre[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar0, b0, tre[s], 0, 0, 0);
        tre[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, b1, tre[s], 0, 0, 0);
        tim[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai0, b0, tim[s], 0, 0, 0);
        tim[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai1, b1, tim[s], 0, 0, 0);
      }
    }
  }
  if (threadIdx.x == 0) {
    dg[n - 1] = s_dii[(n - 1) & 1] * unsc;
    eab[n - 1] = 0.0;
    taus[n - 1] = 0.0;
  }
}

// ------------------------------------------------------ tridiagonal eigen ---
// Number of eigenvalues of the real symmetric tridiagonal (d, e) below x
// (Sturm sequence), restricted to rows [p0, p1].  Exact division.
LRSTV_DEV int sturm_count(const double* dg, const double* e2, int p0, int p1, double x, double pivmin) {
  int cnt = 0;
  double q = dg[p0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = p0 + 1; i <= p1; ++i) {
    q = dg[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// 1/q from the hardware reciprocal refined by one Newton step (full FP64
// accuracy for the normal numbers used here; q is kept away from zero by
// the pivot guards).
LRSTV_DEV double fast_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  return r * (2.0 - q * r);
}

// Same count over the whole matrix with the hardware reciprocal refined by one
// Newton step instead of the full-precision division sequence.
LRSTV_DEV int sturm_count_fast(const double* dg, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = dg[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  // unrolled so that the loads of d and e^2 (the same for every lane) take
  // immediate offsets instead of an address computed per step
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    double rq = __builtin_amdgcn_rcp(q);
    rq = rq * (2.0 - q * rq);  // one Newton step: full FP64 reciprocal accuracy
    q = (dg[i] - x) - e2[i - 1] * rq;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Top-down L D L^T of (T - lk) over rows [p0, p1] (L to column Lp) and the
// twist index minimising gamma_i = (d_i - lk) - u_i e_i - l_{i-1} e_{i-1},
// from the bottom-up U of the same block (column Um) and gamma_p0 = best.
// The u are read 16 rows ahead (rows clamped into the block, unconditional
// loads) and every step is predicated rather than branched, so that the
// loads of the next batch stay in flight across the stores of this one.
LRSTV_DEV int twisted_top(const double* __restrict__ dg, const double* __restrict__ ee,
                          const double* __restrict__ Um, double* __restrict__ Lp, int n, int p0, int p1,
                          double lk, double pivmin, double best) {
  constexpr int PB = 16;
  double dp = dg[p0] - lk;
  if (fabs(dp) < pivmin) dp = pivmin;
  int rt = p0;
  double lkeep = 0.0;
  double v[PB], vn[PB];
  auto load = [&](double (&w)[PB], int i0) {
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int r = i0 + q + 1;
      w[q] = Um[(int64_t)(r < p1 ? r : p1 - 1) * n];
    }
  };
  if (p1 <= p0) return rt;   // a 1 x 1 block: nothing to factor (and no row p1 - 1)
  load(v, p0);
  for (int i0 = p0; i0 < p1; i0 += PB) {
    load(vn, i0 + PB);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int i = i0 + q;
      const bool in = i < p1;
      const int ic = in ? i : p1 - 1;
      const double l = ee[ic] * fast_rcp(dp);
      lkeep = in ? l : lkeep;   // past p1 - 1 the row p1 - 1 is stored again
      Lp[(int64_t)ic * n] = lkeep;
      const double dpr = dg[ic + 1] - lk - l * ee[ic];
      dp = in ? (fabs(dpr) < pivmin ? pivmin : dpr) : dp;
      const double u = i + 1 < p1 ? v[q] : 0.0;
      const double g = fabs(dpr - u * ee[ic + 1]);
      const bool better = in && g < best;
      best = better ? g : best;
      rt = better ? i + 1 : rt;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) v[q] = vn[q];
  }
  return rt;
}

// Column x of a twisted solve with x_rt = 1 over rows [p0, p1] (zero
// outside), from the factors L (rows below the twist) and U (rows above it);
// returns ||x||^2.  The lanes of a wave hold different eigenvalues, with
// their own twist rows and blocks, so both sweeps run over rows common to
// the wave (each lane masking its own range): every load and store of a
// batch then touches one row of 64 consecutive columns.  The downward sweep
// covers every row and stores unconditionally (its value, 1 at the twist, 0
// elsewhere), which also clears the rows outside the block; the upward sweep
// then stores the rows above the twist.  Rows are taken 32 at a time, the
// next batch's loads issued before this batch's stores.
LRSTV_DEV double twisted_solve(const double* __restrict__ Lp, const double* __restrict__ Um, double* __restrict__ x,
                               int n, int p0, int p1, int rt) {
  double nrm = 1.0;
  constexpr int XB = 32;
  double v[XB], xs[XB];
  // rows n-1 down to 0: x_i = -l_i x_{i+1} for p0 <= i < rt
  auto load_l = [&](int i0) {
#pragma unroll
    for (int q = 0; q < XB; ++q) v[q] = Lp[(int64_t)(i0 - q >= 0 ? i0 - q : 0) * n];
  };
  double xv = 1.0;
  int i0 = n - 1;
  load_l(i0);
  while (i0 >= 0) {
#pragma unroll
    for (int q = 0; q < XB; ++q) {
      const int i = i0 - q;
      const bool in = i >= p0 && i < rt;
      const double nx = -v[q] * xv;
      xv = in ? nx : xv;
      nrm += in ? nx * nx : 0.0;
      xs[q] = in ? nx : (i == rt ? 1.0 : 0.0);
    }
    const int b0 = i0;
    i0 -= XB;
    load_l(i0);   // unconditional (past row 0 every row clamps to 0)
    __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the stores
#pragma unroll
    for (int q = 0; q < XB; ++q)
      if (b0 - q >= 0) x[(int64_t)(b0 - q) * n] = xs[q];
  }
  // rows 0 .. n-2 upward: x_{i+1} = -u_i x_i for rt <= i < p1
  auto load_u = [&](int i0) {
#pragma unroll
    for (int q = 0; q < XB; ++q) v[q] = Um[(int64_t)(i0 + q < n - 1 ? i0 + q : n - 2) * n];
  };
  xv = 1.0;
  i0 = 0;
  if (n > 1) load_u(i0);
  while (i0 < n - 1) {
#pragma unroll
    for (int q = 0; q < XB; ++q) {
      const int i = i0 + q;
      const bool in = i >= rt && i < p1;
      const double nx = -v[q] * xv;
      xv = in ? nx : xv;
      nrm += in ? nx * nx : 0.0;
      xs[q] = nx;
    }
    const int b0 = i0;
    i0 += XB;
    load_u(i0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < XB; ++q) {
      const int i = b0 + q;
      if (i >= rt && i < p1) x[(int64_t)(i + 1) * n] = xs[q];
    }
  }
  return nrm;
}

// Counts below xa and below xb over rows [p0, p1], the two recurrences
// interleaved, with the same arithmetic as sturm_count_fast (so that counts
// of blocks add up to its count over the whole matrix).
LRSTV_DEV void sturm_count_pair(const double* dg, const double* e2, int p0, int p1, double xa, double xb,
                                double pivmin, int& ca, int& cb) {
  double qa = dg[p0] - xa, qb = dg[p0] - xb;
  if (fabs(qa) < pivmin) qa = -pivmin;
  if (fabs(qb) < pivmin) qb = -pivmin;
  ca = qa < 0.0;
  cb = qb < 0.0;
  for (int i = p0 + 1; i <= p1; ++i) {
    double ra = __builtin_amdgcn_rcp(qa), rb = __builtin_amdgcn_rcp(qb);
    ra = ra * (2.0 - qa * ra);
    rb = rb * (2.0 - qb * rb);
    qa = (dg[i] - xa) - e2[i - 1] * ra;
    qb = (dg[i] - xb) - e2[i - 1] * rb;
    if (fabs(qa) < pivmin) qa = -pivmin;
    if (fabs(qb) < pivmin) qb = -pivmin;
    ca += qa < 0.0;
    cb += qb < 0.0;
  }
}

// Threads per eigenvalue in the eigenvalue phase (interior probe points of
// each section step): 2 where the launch gives at least two waves per SIMD
// (the phase is then bound by FP64 issue, and trisection needs the fewest
// counts: about 22 rounds of 2 from the grid cell), 4 for smaller launches
// (5-section, 15 rounds of 4).  Measured at 256x256x191: 0.60 -> 0.55 ms for
// the 256-slice launch with 2; the 32 slices run beside the other group's
// kernels and share its CUs, so fewer rounds at more counts did not pay
// there (8 probes: 0.37 -> 1.10 ms).
static int device_cus();
static int eig_probes(int ns, int n) {
  const long long waves2 = (long long)ns * n * 2 / 64;
  const int simds = 4 * device_cus();
  return waves2 >= 2 * simds ? 2 : 4;
}

// Eigenvalues above (t^2 - delta) of T / ||T|| by multisection (2 or 4
// threads per eigenvalue, blocks of 256 threads), eigenvectors by twisted
// factorisation inside their unreduced block, Gram-Schmidt inside clusters;
// output column c = eigenvector of the c-th largest kept eigenvalue times the
// phase (V re/im planes).
// PHASE 0 computes the eigenvalues (kept in the tridiagonal scratch at 5n,
// scaled by 1 / ||T||); PHASE 1 the eigenvectors from them, spread over
// blocks of 64 eigenvalues (grid: vector blocks x slices), so that more
// waves hide the latency of their sequential recurrences; PHASE 2
// normalises them, re-orthogonalises clusters and writes V.  Each redoes the
// O(n) set-up (scaling, splits); PHASE 0 also counts the eigenvalues below
// the cut and publishes the rank, which the later phases read back.
template <int PHASE>
__global__ void __launch_bounds__(PHASE == 1 ? 64 : (PHASE == 0 ? 256 : 1024)) k_trieig(const SliceDesc* __restrict__ desc, double* __restrict__ tri,
                                                 double* __restrict__ xs, float* __restrict__ V,
                                                 int* __restrict__ rcount, const double* __restrict__ mu_dev,
                                                 double alpha, float thresh, int probes, const int* __restrict__ halt) {
  extern __shared__ double smd[];
  __shared__ double red[16];
  __shared__ int s_c0, s_nblk;
  // PHASES 0 and 1 run a grid of (eigenvalue blocks, slices), PHASE 2 one
  // block per slice
  const int slice = PHASE == 2 ? blockIdx.x : blockIdx.y;
  const SliceDesc d = desc[slice];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1;
  double* dg = tri + d.t_off;
  const double* eab = dg + n;
  const double* phr = eab + n;
  const double* phi = phr + n;
  double* e2 = smd;                 // [n]
  double* ee = e2 + n;              // [n] off-diagonal with splits zeroed
  double* lam = ee + n;             // [n]
  double* ds = lam + n;             // [n] diagonal
  double* sdot = ds + n;            // [n] Gram-Schmidt coefficients
  int* bstart = (int*)(sdot + n);   // [n+1] block starts
  int* gcnt = bstart + n + 1;       // [blockDim] eigenvalue counts on the coarse grid
  const double t = mu_dev ? alpha / *mu_dev : (double)thresh;
  double gl = 1e300, gu = -1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double e = (i < n - 1) ? eab[i] : 0.0;
    if (i < n - 1 && e <= 1e-15 * (fabs(dg[i]) + fabs(dg[i + 1]))) e = 0.0;
    ee[i] = e;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double rad = ee[i] + (i > 0 ? ee[i - 1] : 0.0);
    gl = fmin(gl, dg[i] - rad);
    gu = fmax(gu, dg[i] + rad);
  }
  gl = -block_max(-gl, red);
  gu = block_max(gu, red);
  const double tnorm0 = fmax(fabs(gl), fabs(gu));
  // work on T / ||T|| so that the pivot guards stay far from overflow
  const double sc = tnorm0 > 0.0 ? 1.0 / tnorm0 : 1.0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    ds[i] = dg[i] * sc;
    ee[i] *= sc;
    e2[i] = ee[i] * ee[i];
  }
  gl *= sc;
  gu *= sc;
  __syncthreads();
  const double tnorm = tnorm0 > 0.0 ? 1.0 : 0.0;
  const double pivmin = 1e-290;
  const double delta = 1e-6 * tnorm;                    // FP32 resolution of the Gram
  // thresh < 0 without a device mu asks for every eigenpair (the t-SVT
  // derivative needs the full spectrum)
  const bool all = (mu_dev == nullptr && thresh < 0.f) || d.keep > 0;
  const double lo_cut = all ? gl - 1.0 : fmax(t * t * sc - delta, 0.0);
  dg = ds;
  // unreduced blocks (starts after each zero off-diagonal) by a ballot scan
  // in the first wave, and the count of eigenvalues below the cut
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int nb = 1;
    for (int i0 = 0; i0 < n - 1; i0 += 64) {
      const int i = i0 + lane;
      const bool split = i < n - 1 && ee[i] == 0.0;
      const unsigned long long m = __ballot(split);
      if (split) bstart[nb + __popcll(m & ((1ull << lane) - 1ull))] = i + 1;
      nb += __popcll(m);
    }
    if (lane == 0) {
      bstart[0] = 0;
      bstart[nb] = n;
      s_nblk = nb;
      // the count below the cut: computed once per slice by the eigenvalue
      // phase, which publishes r = n - c0 in rcount (the kernels after the
      // eigen-solve read the rank there); the later phases take it back
      if (PHASE == 0) {
        const int c0v = d.keep > 0 ? n - (d.keep < n ? d.keep : n)
                      : all ? 0 : (tnorm == 0.0) ? n : sturm_count_fast(dg, e2, n, lo_cut, pivmin);
        s_c0 = c0v;
        if (blockIdx.x == 0) rcount[slice] = n - c0v;
      } else {
        s_c0 = n - rcount[slice];
      }
    }
  }
  __syncthreads();
  const int c0 = s_c0, nblk = s_nblk, r = n - c0;
  double* lam_g = tri + d.t_off + 5 * n;   // eigenvalues between the two phases
  if (PHASE != 0) {
    for (int k = c0 + threadIdx.x; k < n; k += blockDim.x) lam[k] = lam_g[k];
  }
  // Shared first step: the counts at G = blockDim points spread over
  // [lo0, gu] bracket every eigenvalue in one grid cell.  Then
  // (probes + 1)-section: the probes threads of a group probe as many
  // interior points of the cell, until it is below max(eps_64 |lambda|,
  // 1e-13 ||T||) (the FP32 Gram resolves its eigenvalues to ~1e-7 ||T||;
  // clusters are gaps below 1e-10 ||T||); probes from eig_probes.
  if (PHASE == 0) {
    // block x takes the eigenvalues c0 + [E x, E x + E), E = blockDim /
    // probes (and every gridDim.x * E-th block of them beyond), so that a
    // slice's work spreads over several CUs and the launch balances around
    // busy ones
    const int PR = probes;
    const int G = blockDim.x, ngrp = blockDim.x / PR, stride = ngrp * gridDim.x;
    if (blockIdx.x * ngrp >= r) return;
    const double lo0 = fmax(gl, lo_cut), cell = (gu - lo0) / G;
    gcnt[threadIdx.x] = sturm_count_fast(dg, e2, n, lo0 + (threadIdx.x + 1) * cell, pivmin);
    __syncthreads();
    const int lane = threadIdx.x & 63, q = lane % PR, base = lane - q;
    const int nround = (r - blockIdx.x * ngrp + stride - 1) / stride;
    for (int rd = 0; rd < nround; ++rd) {
      const int kk = threadIdx.x / PR + blockIdx.x * ngrp + rd * stride;
      const bool act = kk < r;
      const int k = c0 + kk;
      // first grid point whose count exceeds k: lambda_k in [x_{j-1}, x_j)
      int jl = 0, jh = G;
      while (jl < jh) {
        const int mid = (jl + jh) >> 1;
        if (gcnt[mid] > k) jh = mid;
        else jl = mid + 1;
      }
      double lo = lo0 + jl * cell, hi = lo0 + (jl + 1) * cell;
      for (int it = 0; it < 128; ++it) {
        const double wdt = hi - lo;
        const bool done = !act || wdt <= fmax(2.2e-16 * fmax(fabs(lo), fabs(hi)), 1e-13 * tnorm);
        if (__all(done)) break;
        const double step = wdt * (1.0 / (PR + 1));
        const double x = lo + (q + 1) * step;
        const int cnt = done ? 0 : sturm_count_fast(dg, e2, n, x, pivmin);
        // eigenvalue k lies in the first section whose upper count exceeds k
        int j = PR;
        for (int pp = PR - 1; pp >= 0; --pp)
          if (__shfl(cnt, base + pp, 64) > k) j = pp;
        if (!done) {
          const double nlo = lo + j * step;
          hi = j < PR ? lo + (j + 1) * step : hi;
          lo = nlo;
        }
      }
      // The value stored is canonical, independent of the search path (the
      // probe count follows the launch size, and a cube must give the same
      // result alone and in a batch): the midpoint of the cell of a fixed
      // lattice of spacing h = 2^-43 ||T|| (above the stopping width, so
      // that [lo, hi] holds at most one lattice point) that holds the
      // eigenvalue, the cell decided by the count at that point.
      const double h = 0x1p-43;   // T is scaled to ||T|| = 1
      double cl = floor(lo / h) * h;
      const double g = cl + h;
      const bool gin = act && g <= hi;
      const int cg = gin ? sturm_count_fast(dg, e2, n, g, pivmin) : 0;
      if (gin && cg <= k) cl = g;   // lambda_k >= g
      if (act && q == 0) lam_g[k] = cl + 0.5 * h;
    }
    return;
  }
  __syncthreads();
  // eigenvectors: twisted factorisation, one eigenvalue per thread
  const int64_t nn = (int64_t)n * n;
  double* X = xs + d.x_off;    // [3][n][n] : Um, Dm(-> x), Lp ; column index k - c0
  const double tol_eq = 1e-13 * tnorm + pivmin;
  if (PHASE == 2) goto reorth;
  for (int k = c0 + blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int col = k - c0;
    const double lk = lam[k];
    int pick = 0;
    if (nblk > 1) {
      // locate the unreduced block that holds this copy of lk: the count
      // below lk - tol over the whole matrix is the sum of the blocks'
      // counts (the recurrence restarts exactly where e^2 = 0), then the
      // blocks' counts at lk -+ tol (two interleaved recurrences) until the
      // copy is reached
      int m = k - sturm_count_fast(dg, e2, n, lk - tol_eq, pivmin);
      for (int b = 0; b < nblk; ++b) {
        int clo, chi;
        sturm_count_pair(dg, e2, bstart[b], bstart[b + 1] - 1, lk - tol_eq, lk + tol_eq, pivmin, clo, chi);
        const int eq = chi - clo;
        if (eq > 0) {
          pick = b;
          if (m < eq) break;
          m -= eq;
        }
      }
    }
    const int p0 = bstart[pick], p1 = bstart[pick + 1] - 1;
    double* Um = X + col;
    double* Dm = X + nn + col;
    double* Lp = X + 2 * nn + col;
    // bottom-up U D U^T (only U is stored: the twist criterion below is
    // formed from U and L)
    double dm = dg[p1] - lk;
    if (fabs(dm) < pivmin) dm = pivmin;
#pragma unroll 4
    for (int i = p1 - 1; i >= p0; --i) {
      const double u = ee[i] * fast_rcp(dm);
      Um[(int64_t)i * n] = u;
      dm = dg[i] - lk - u * ee[i];
      if (fabs(dm) < pivmin) dm = pivmin;
    }
    // top-down L D L^T and twist index: gamma_i = dm_i + dp_i - (d_i - lk)
    // = (d_i - lk) - u_i e_i - l_{i-1} e_{i-1} (gamma_p0 = dm_p0, and no u
    // term at p1)
    const int rt = twisted_top(dg, ee, Um, Lp, n, p0, p1, lk, pivmin, fabs(dm));
    // solve with the twist: x_rt = 1
    double* x = Dm;
    const double nrm = twisted_solve(Lp, Um, x, n, p0, p1, rt);
    // the vector stays unscaled here: 1 / ||x|| goes to the first row of the
    // (no longer needed) U scratch, and PHASE 2 scales all columns at once
    // (a per-thread pass over its own column would serialise on the global
    // loads)
    Um[0] = 1.0 / sqrt(nrm);
  }
  if (PHASE == 1) return;
reorth:
  __syncthreads();
  // Re-orthogonalise inside clusters (gaps below 1e-10 ||T||; larger gaps give
  // FP64 twisted-factorisation vectors accurate to eps_64 / gap): classical
  // Gram-Schmidt applied twice per vector against the earlier cluster members.
  // That needs the normalised vectors in place; a slice without a cluster
  // (the usual case) applies the scale while V is written instead, one pass
  // over the vectors instead of three.
  double* Xv = X + nn;
  const double gtol = 1e-10 * tnorm;
  __shared__ int s_cluster;
  if (threadIdx.x == 0) s_cluster = 0;
  __syncthreads();
  for (int k = c0 + 1 + threadIdx.x; k < n; k += blockDim.x)
    if (lam[k] - lam[k - 1] <= gtol) s_cluster = 1;
  __syncthreads();
  const bool cluster = s_cluster != 0;
  constexpr int U8 = 8;
  if (cluster) {
    const int tot = n * r;
    for (int e0 = threadIdx.x; e0 < tot; e0 += U8 * blockDim.x) {
      double v[U8];
      int64_t ofs[U8];
#pragma unroll
      for (int u = 0; u < U8; ++u) {
        const int e = e0 + u * blockDim.x;
        ofs[u] = -1;
        if (e < tot) {
          const int i = e / r, c = e - i * r;
          ofs[u] = (int64_t)i * n + c;
          v[u] = Xv[ofs[u]] * X[c];
        }
      }
#pragma unroll
      for (int u = 0; u < U8; ++u)
        if (ofs[u] >= 0) Xv[ofs[u]] = v[u];
    }
    __syncthreads();
    for (int k = c0 + 1; k < n; ++k) {
      int k0 = k;
      while (k0 > c0 && lam[k0] - lam[k0 - 1] <= gtol) --k0;
      if (k0 == k) continue;
      const int ck = k - c0, cb = k0 - c0, nc = k - k0;
      for (int pass = 0; pass < 2; ++pass) {
        // one wave per coefficient, its lanes over the rows
        {
          const int lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
          for (int j = threadIdx.x >> 6; j < nc; j += nwv) {
            double dt = 0.0;
            for (int i = lane; i < n; i += 64) dt += Xv[(int64_t)i * n + cb + j] * Xv[(int64_t)i * n + ck];
            dt = wave_sum_dpp(dt);
            if (lane == 0) sdot[j] = dt;
          }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
          double acc = 0.0;
          for (int j = 0; j < nc; ++j) acc += sdot[j] * Xv[(int64_t)i * n + cb + j];
          Xv[(int64_t)i * n + ck] -= acc;
        }
        __syncthreads();
      }
      double nr = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) nr += Xv[(int64_t)i * n + ck] * Xv[(int64_t)i * n + ck];
      nr = block_sum(nr, red);
      const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) Xv[(int64_t)i * n + ck] *= inv;
      __syncthreads();
    }
  }
  // V[:, c] = phase .* x for the c-th largest eigenvalue (times 1 / ||x||
  // when it was not applied above).  A thread keeps one column (its scale
  // loaded once) and every (blockDim / 256)-th row, eight loads in flight;
  // the phases are staged in LDS (e^2 and e are no longer needed).
  float* Vr = V + d.v_off;
  float* Vi = Vr + nn;
  double* sphr = e2;
  double* sphi = ee;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    sphr[i] = phr[i];
    sphi[i] = phi[i];
  }
  __syncthreads();
  const int ngr = blockDim.x >> 8;
  for (int cb0 = 0; cb0 < r; cb0 += 256) {
    const int c = cb0 + (threadIdx.x & 255);
    if (c >= r) continue;
    const int col = n - 1 - c - c0;
    const double scl = cluster ? 1.0 : X[col];
    for (int i0 = threadIdx.x >> 8; i0 < n; i0 += U8 * ngr) {
      double xv[U8];
#pragma unroll
      for (int u = 0; u < U8; ++u) {
        const int i = i0 + u * ngr;
        xv[u] = i < n ? Xv[(int64_t)i * n + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U8; ++u) {
        const int i = i0 + u * ngr;
        if (i < n) {
          const double x = cluster ? xv[u] : xv[u] * scl;
          Vr[(int64_t)i * n + c] = (float)(sphr[i] * x);
          Vi[(int64_t)i * n + c] = (float)(sphi[i] * x);
        }
      }
    }
  }
  if (threadIdx.x == 0) rcount[slice] = r;
}

// ------------------------------------------- blocked back-transform (WY) ---
// V <- H_0 H_1 ... H_{n-2} V with the reflectors grouped 64 at a time:
// H_{i0} ... H_{i0+63} = I - Y T Y^H (Y: the block's reflectors as columns,
// T upper triangular, T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] Y^H y_j),
// applied from the last block to the first as V -= Y (T (Y^H V)), three
// complex products on the matrix cores per block.

// Y(k, p) of the block starting at reflector i0: matrix row i0 + 1 + k,
// reflector i0 + p (zero above its leading 1 and past the last reflector).
LRSTV_DEV float2 wy_y(const float2* __restrict__ g, int n, int i0, int nbk, int k, int p) {
  const int row = i0 + 1 + k;
  if (p >= nbk || row >= n || k < p) return make_float2(0.f, 0.f);
  return g[packed(row, i0 + p)];
}

// T factor of one reflector block (placed by xcd_tile_slice over
// (reflector block, slice), so that the blocks of a slice share an L2).
__global__ void __launch_bounds__(256) k_wy_t(const SliceDesc* __restrict__ desc, const float2* __restrict__ gram,
                                              const double* __restrict__ tri, float* __restrict__ Twy,
                                              const int* __restrict__ rcount, int ntile, int ns, const int* __restrict__ halt) {
  // one LDS buffer (40 KB, four blocks per CU): the product's staging, then
  // S = Y^H Y and the in-place inversion (T below)
  __shared__ MfmaSmem sm;
  float2(*T)[65] = reinterpret_cast<float2(*)[65]>(&sm);
  static_assert(sizeof(MfmaSmem) >= 64 * 65 * sizeof(float2), "T factor scratch");
  int b, slice;
  if (!xcd_tile_slice(ntile, ns, b, slice)) return;
  const SliceDesc d = desc[slice];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1, nblk = (n - 1 + 63) / 64;
  if (b >= nblk || rcount[slice] == 0) return;
  const int i0 = 64 * b, m = n - 1 - i0, nbk = m < 64 ? m : 64;
  const float2* g = gram + d.g_off;
  const double* taus = tri + d.t_off + 4 * n;
  // S = Y^H Y
  auto fa = [&](int p, int k) -> float2 {
    const float2 y = (k < m) ? wy_y(g, n, i0, nbk, k, p) : make_float2(0.f, 0.f);
    return make_float2(y.x, -y.y);
  };
  auto fb = [&](int k, int q) -> float2 { return (k < m) ? wy_y(g, n, i0, nbk, k, q) : make_float2(0.f, 0.f); };
  // the stores come after the product's last barrier, so S may overwrite
  // the staging buffer
  auto st = [&](int p, int q, float2 v) { T[p][q] = v; };
  mfma_ctile<kF32, false, false>(0, 0, m, fa, fb, st, sm, true);
  __syncthreads();
  // T from its inverse: for reflectors I - tau_j y_j y_j^H, T^-1 =
  // diag(1 / tau) + (strict upper part of Y^H Y) (the compact-WY identity of
  // Puglisi, and of Joffrain, Low, Quintana-Orti, van de Geijn and van Zee).
  // The upper triangular inverse by doubling: with the inverses of two
  // adjacent diagonal blocks A and C of size s known, the block between them
  // is -A B C (B the block of the inverse's argument), six levels of small
  // products instead of a 64-step sequential recurrence.  A reflector with
  // tau = 0 (or past the block's last) has a zero column in Y: its diagonal
  // entry is 1 during the inversion (its off-diagonal entries are zero) and
  // 0 in the result.  The inversion runs in place: the strict upper part of
  // T holds the argument's blocks B until the level that replaces them by
  // -A B C, the diagonal holds the inverses tau_j, and the products B C go to
  // the (free) mirrored lower block, transposed.  Rows are padded to 65 so
  // that neither the row-wise nor the column-wise accesses conflict in the
  // LDS banks.
  for (int p = threadIdx.x; p < 64; p += blockDim.x) {
    const float tp = p < nbk ? (float)taus[i0 + p] : 0.f;
    T[p][p] = make_float2(tp != 0.f ? tp : 1.f, 0.f);
  }
  __syncthreads();
  for (int s2 = 1; s2 < 64; s2 <<= 1) {
    const int E = 32 * s2;   // (32 / s2) block pairs of s2 x s2 entries
    // M = B C, stored as T[b1 + c][b0 + r] = M(r, c)
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
      const int pr = e / (s2 * s2), rem = e - pr * s2 * s2, r = rem / s2, c = rem - r * s2;
      const int b0 = 2 * s2 * pr, b1 = b0 + s2;
      float2 acc = make_float2(0.f, 0.f);
      for (int k = 0; k <= c; ++k) acc = cadd(acc, cmul(T[b0 + r][b1 + k], T[b1 + k][b1 + c]));
      T[b1 + c][b0 + r] = acc;
    }
    __syncthreads();
    // X = -A M into the upper block of T
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
      const int pr = e / (s2 * s2), rem = e - pr * s2 * s2, r = rem / s2, c = rem - r * s2;
      const int b0 = 2 * s2 * pr, b1 = b0 + s2;
      float2 acc = make_float2(0.f, 0.f);
      for (int k = r; k < s2; ++k) acc = cadd(acc, cmul(T[b0 + r][b0 + k], T[b1 + c][b0 + k]));
      T[b0 + r][b1 + c] = make_float2(-acc.x, -acc.y);
    }
    __syncthreads();
  }
  // stored transposed: T(p, q) at q * 64 + p
  float* out = Twy + d.y_off + (int64_t)b * 64 * 64 * 2;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int q = e >> 6, p = e & 63;
    float2 t = p <= q ? T[p][q] : make_float2(0.f, 0.f);
    if (p == q && !(p < nbk && taus[i0 + p] != 0.0)) t = make_float2(0.f, 0.f);
    out[e] = t.x;
    out[64 * 64 + e] = t.y;
  }
}

// One column tile (64 columns of V) of a slice, placed by xcd_tile_slice
// over (column tile, slice): every reflector block, last to first, on the
// same columns, as
//   W = Y^H V,  W' = T W,  V -= Y W'.
// Wave q owns the 16 columns 16 q .. 16 q + 15 and keeps W and W' (64 x 16
// complex) in the accumulators of v_mfma_f32_16x16x4f32: element r of lane l
// of row tile t is row 16 t + 4 (l / 16) + r, column l % 16, which is exactly
// the B operand (row l / 16, column l % 16) of the step that contracts over
// the rows {16 t + 4 g + r, g = 0..3}.  So W and W' never leave the registers;
// only the operands Y, T and V are staged through LDS, shared by the four
// waves, in chunks of 32 rows with the next chunk's loads in flight (one
// loader for both passes over V).  The last product is added into the
// staged V, which is written back coalesced.  LDS row strides are chosen so
// that the operand reads are free of bank conflicts: 80 where a lane's row
// is 4 s + l / 16 (16 (l / 16) + l % 16 distinct mod 64), 68 and 36 where it
// is 16 t + 4 (l / 16) + r (16 (l / 16) + l % 16 again).
struct WySmem {
  union {
    struct {
      float yr[32][80], yi[32][80], vr[32][80], vi[32][80];   // Y(k, p), V(k, c), k in the chunk
    } a;
    struct {
      float tr[64][68], ti[64][68];                           // T(p, q) at [q][p]
    } t;
    struct {
      float yr[64][36], yi[64][36];                           // Y(k, p) at [p][k], k in the chunk
      float vr[32][68], vi[32][68];                           // V(k, c)
    } u;
  };
};

__global__ void __launch_bounds__(256, 3) k_wy_apply(const SliceDesc* __restrict__ desc, const float2* __restrict__ gram,
                                                     const float* __restrict__ Twy, float* __restrict__ V,
                                                     const int* __restrict__ rcount, int ntile, int ns, const int* __restrict__ halt) {
  __shared__ WySmem sm;
  int ct, slice;
  if (!xcd_tile_slice(ntile, ns, ct, slice)) return;
  const SliceDesc d = desc[slice];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int n = d.n1, r = rcount[slice], c0 = 64 * ct;
  if (c0 >= r) return;
  const int nc = (r - c0) < 64 ? (r - c0) : 64;
  const int nblk = (n - 1 + 63) / 64;
  const float2* g = gram + d.g_off;
  float* Vr = V + d.v_off;
  float* Vi = Vr + (int64_t)n * n;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 15, lg = lane >> 4;
  const int ccol = 16 * wv + li;       // this lane's column within the tile
  const bool act = 16 * wv < nc;       // wave-uniform: the wave has columns to update
  for (int b = nblk - 1; b >= 0; --b) {
    const int i0 = 64 * b, m = n - 1 - i0, nbk = m < 64 ? m : 64;
    // ---- W = Y^H V[i0+1:, cols]: chunks of 32 rows, staged with the next
    // chunk's loads in flight.  Staged element e = t + 256 j: row e / 64,
    // column e % 64 (coalesced along the row).
    // three real products per complex one (3M): with A = conj(Y), P1 = Yr Vr,
    // P2 = Yi Vi, P3 = (Yr - Yi)(Vr + Vi); Re W = P1 + P2, Im W = P3 - P1 + P2
    f32x4 w1[4], w2[4], w3[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w1[q] = w2[q] = w3[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    float2 ys[8], vs[8];
    auto load1 = [&](int k0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = t + 256 * j, kk = e >> 6, cc = e & 63, k = k0 + kk;
        ys[j] = k < m ? wy_y(g, n, i0, nbk, k, cc) : make_float2(0.f, 0.f);
        vs[j] = make_float2(0.f, 0.f);
        if (k < m && cc < nc) {
          const int64_t q = (int64_t)(i0 + 1 + k) * n + c0 + cc;
          vs[j] = make_float2(Vr[q], Vi[q]);
        }
      }
    };
    load1(0);
    for (int k0 = 0; k0 < m; k0 += 32) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = t + 256 * j, kk = e >> 6, cc = e & 63;
        sm.a.yr[kk][cc] = ys[j].x;
        sm.a.yi[kk][cc] = ys[j].y;
        sm.a.vr[kk][cc] = vs[j].x;
        sm.a.vi[kk][cc] = vs[j].y;
      }
      __syncthreads();
      if (k0 + 32 < m) load1(k0 + 32);
      if (act) {
#pragma unroll 1
        for (int s = 0; s < 8; ++s) {
          const int kk = 4 * s + lg;
          const float br = sm.a.vr[kk][ccol], bi = sm.a.vi[kk][ccol], bs = br + bi;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float ar = sm.a.yr[kk][16 * q + li], ai = sm.a.yi[kk][16 * q + li];
            w1[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, w1[q], 0, 0, 0);
            w2[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, w2[q], 0, 0, 0);
            w3[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar - ai, bs, w3[q], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
    f32x4 wr[4], wi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wr[q] = w1[q] + w2[q];
      wi[q] = w3[q] - w1[q] + w2[q];
    }
    // ---- W' = T W (T upper triangular: row tile p of W' takes row tiles
    // q >= p of W).  T is stored transposed, T(p, q) at [q][p].  3M again:
    // P1 = Tr Wr, P2 = Ti Wi, P3 = (Tr + Ti)(Wr + Wi).
    {
      const float* Tt = Twy + d.y_off + (int64_t)b * 64 * 64 * 2;
#pragma unroll 4
      for (int j = 0; j < 16; ++j) {
        const int e = t + 256 * j;
        sm.t.tr[e >> 6][e & 63] = Tt[e];
        sm.t.ti[e >> 6][e & 63] = Tt[64 * 64 + e];
      }
    }
    __syncthreads();
    f32x4 x1[4], x2[4], x3[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x1[q] = x2[q] = x3[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (act) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = 16 * q + 4 * lg + rr;
          const float br = wr[q][rr], bi = wi[q][rr], bs = br + bi;
#pragma unroll
          for (int p = 0; p <= q; ++p) {
            const float ar = sm.t.tr[row][16 * p + li], ai = sm.t.ti[row][16 * p + li];
            x1[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, x1[p], 0, 0, 0);
            x2[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, x2[p], 0, 0, 0);
            x3[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar + ai, bs, x3[p], 0, 0, 0);
          }
          // keep the operand reads of one row step together (register budget)
          __builtin_amdgcn_sched_barrier(0);
        }
    }
    f32x4 xr[4], xi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xr[q] = x1[q] - x2[q];
      xi[q] = x3[q] - x1[q] - x2[q];
    }
    __syncthreads();
    // ---- V[i0+1:, cols] -= Y W': chunks of 32 rows; 3M with P1 = Yr W'r,
    // P2 = Yi W'i, P3 = (Yr + Yi)(W'r + W'i).
    load1(0);
    for (int k0 = 0; k0 < m; k0 += 32) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = t + 256 * j, kk = e >> 6, cc = e & 63;
        sm.u.yr[cc][kk] = ys[j].x;
        sm.u.yi[cc][kk] = ys[j].y;
        sm.u.vr[kk][cc] = vs[j].x;
        sm.u.vi[kk][cc] = vs[j].y;
      }
      __syncthreads();
      if (k0 + 32 < m) load1(k0 + 32);
      if (act) {
        f32x4 u1[2], u2[2], u3[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) u1[kt] = u2[kt] = u3[kt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int p = 16 * q + 4 * lg + rr;
            const float br = xr[q][rr], bi = xi[q][rr], bs = br + bi;
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
              const float ar = sm.u.yr[p][16 * kt + li], ai = sm.u.yi[p][16 * kt + li];
              u1[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, u1[kt], 0, 0, 0);
              u2[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, u2[kt], 0, 0, 0);
              u3[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar + ai, bs, u3[kt], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        // element rr of lane l of row tile kt: row 16 kt + 4 (l / 16) + rr
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = 16 * kt + 4 * lg + rr;
            sm.u.vr[row][ccol] -= u1[kt][rr] - u2[kt][rr];
            sm.u.vi[row][ccol] -= u3[kt][rr] - u1[kt][rr] - u2[kt][rr];
          }
      }
      __syncthreads();
      // each thread writes back the elements it staged (the next staging
      // overwrites only those, so no barrier is needed before it)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = t + 256 * j, kk = e >> 6, cc = e & 63, k = k0 + kk;
        if (k < m && cc < nc) {
          const int64_t q = (int64_t)(i0 + 1 + k) * n + c0 + cc;
          Vr[q] = sm.u.vr[kk][cc];
          Vi[q] = sm.u.vi[kk][cc];
        }
      }
    }
    __syncthreads();
  }
}

void launch_backtrans(const SvtLaunch& L, hipStream_t s) {
  const int n = L.max_n1, ns = L.n_slices;
  const int nblk = (n - 1 + 63) / 64;
  if (nblk == 0 || ns == 0) return;
  hipLaunchKernelGGL(k_wy_t, dim3(xcd_grid(nblk, ns)), dim3(256), 0, s, L.desc, L.gram, L.tri, L.Twy, L.rcount, nblk,
                     ns, L.halt);
  const int ncb = (n + 63) / 64;
  hipLaunchKernelGGL(k_wy_apply, dim3(xcd_grid(ncb, ns)), dim3(256), 0, s, L.desc, L.gram, L.Twy, L.V, L.rcount, ncb,
                     ns, L.halt);
}

// ----------------------------------------------------- back-projection ---
// tall: B (h x r, ld n) = M V_r;  wide: B (r x w, ld w) = U_r^H M
template <int MODE>
__global__ void __launch_bounds__(256) k_bp1(const SliceDesc* __restrict__ desc, const float* __restrict__ sl,
                                             const float* __restrict__ V, float* __restrict__ Bb,
                                             const int* __restrict__ rcount, int tdim, int ns, const int* __restrict__ halt) {
  __shared__ MfmaSmem sm;
  int tile, slice;
  if (!xcd_tile_slice(tdim * tdim, ns, tile, slice)) return;
  const int bx = tile % tdim, by = tile / tdim;
  const SliceDesc d = desc[slice];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int r = rcount[slice], n = d.n1, h = d.h, w = d.w;
  const float* mr = sl + d.a_off;
  const float* mi = mr + (int64_t)h * w;
  const float* vr = V + d.v_off;
  const float* vi = vr + (int64_t)n * n;
  float* br = Bb + d.b_off;
  float* bi = br + (int64_t)h * w;
  const int m0 = by * kMT, n0 = bx * kMT;
  const int M = d.tall ? h : r, N = d.tall ? r : w, ld = d.tall ? n : w;
  if (m0 >= M || n0 >= N) return;
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < M && n0 + 32 * (wv & 1) < N;
  auto st = [&](int a, int b, float2 v) {
    if (a < M && b < N) { br[(int64_t)a * ld + b] = v.x; bi[(int64_t)a * ld + b] = v.y; }
  };
  if (d.tall) {
    auto fa = [&](int m, int k0, float2(&v)[8]) {
      const int nv = m < h ? w - k0 : 0;
      float a[8], b[8];
      load8(mr + (int64_t)m * w + k0, nv, a);
      load8(mi + (int64_t)m * w + k0, nv, b);
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = make_float2(a[j], b[j]);
    };
    auto fb = [&](int k, int c) -> float2 {
      if (k >= n || c >= r) return make_float2(0.f, 0.f);
      return make_float2(vr[(int64_t)k * n + c], vi[(int64_t)k * n + c]);
    };
    mfma_ctile<MODE, true, false, true, false>(m0, n0, w, fa, fb, st, sm, active);
  } else {
    auto fa = [&](int m, int k) -> float2 {
      if (m >= r || k >= h) return make_float2(0.f, 0.f);
      return make_float2(vr[(int64_t)k * n + m], -vi[(int64_t)k * n + m]);
    };
    auto fb = [&](int k, int c) -> float2 {
      if (k >= h || c >= w) return make_float2(0.f, 0.f);
      return make_float2(mr[(int64_t)k * w + c], mi[(int64_t)k * w + c]);
    };
    mfma_ctile<MODE, false, false>(m0, n0, h, fa, fb, st, sm, active);
  }
}

// sigma_c = ||B[:, c]|| (tall) or ||B[c, :]|| (wide); f_c = max(1 - t/sigma_c, 0)
__global__ void __launch_bounds__(256) k_colnorm(const SliceDesc* __restrict__ desc, const float* __restrict__ Bb,
                                                 float* __restrict__ fval, const int* __restrict__ rcount,
                                                 const double* __restrict__ mu_dev, double alpha, float thresh, const int* __restrict__ halt) {
  // Block (x, slice) takes the singular indices 64 x .. 64 x + 63; squares
  // are summed in FP64.  Tall: B is h x r at row stride n, thread t takes
  // column 64 x + t % 64 and rows t / 64 + 4 j, so each row read of a wave is
  // 64 consecutive floats.  Wide: B is r x w, wave q takes the rows
  // 64 x + 16 q .. + 15, one contiguous row at a time.
  __shared__ double part[4][64];
  const SliceDesc d = desc[blockIdx.y];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int r = rcount[blockIdx.y], c0 = 64 * blockIdx.x;
  if (c0 >= r) return;
  const int h = d.h, w = d.w, n = d.n1;
  const float* br = Bb + d.b_off;
  const float* bi = br + (int64_t)h * w;
  const double t = mu_dev ? alpha / *mu_dev : (double)thresh;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  auto shrink = [&](double s2) {
    const double sg = sqrt(s2);
    return (sg > t) ? (float)(1.0 - t / sg) : 0.f;
  };
  if (d.tall) {
    const int c = c0 + lane;
    double s = 0.0;
    if (c < r) {
#pragma unroll 8
      for (int i = wv; i < h; i += 4) {
        const double a = br[(int64_t)i * n + c], b = bi[(int64_t)i * n + c];
        s += a * a + b * b;
      }
    }
    part[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && c < r) fval[d.f_off + c] = shrink(part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
  } else {
    for (int cc = 0; cc < 16; ++cc) {
      const int c = c0 + 16 * wv + cc;
      if (c >= r) break;  // wave-uniform
      double s = 0.0;
      for (int i = lane; i < w; i += 64) {
        const double a = br[(int64_t)c * w + i], b = bi[(int64_t)c * w + i];
        s += a * a + b * b;
      }
      s = warp_sum(s);
      if (lane == 0) fval[d.f_off + c] = shrink(s);
    }
  }
}

// tall: Ehat (h x w) = B diag(f) V_r^H;  wide: Ehat = U_r diag(f) B.  Written over M.
template <int MODE>
__global__ void __launch_bounds__(256, MODE == kF32 ? 4 : 1) k_bp2(const SliceDesc* __restrict__ desc, float* __restrict__ sl,
                                             const float* __restrict__ V, const float* __restrict__ Bb,
                                             const float* __restrict__ fval, const int* __restrict__ rcount, int tdim,
                                             int ns, const int* __restrict__ halt) {
  __shared__ MfmaSmem sm;
  int tile, slice;
  if (!xcd_tile_slice(tdim * tdim, ns, tile, slice)) return;
  const int bx = tile % tdim, by = tile / tdim;
  const SliceDesc d = desc[slice];
  if (d.prio) __builtin_amdgcn_s_setprio(3);   // the later group's chain issues first
  if (halt && halt[d.cube]) return;   // the cube has met its stopping test
  const int r = rcount[slice], n = d.n1, h = d.h, w = d.w;
  const int m0 = by * kMT, n0 = bx * kMT;
  if (m0 >= h || n0 >= w) return;
  float* er = sl + d.a_off;
  float* ei = er + (int64_t)h * w;
  const float* vr = V + d.v_off;
  const float* vi = vr + (int64_t)n * n;
  const float* br = Bb + d.b_off;
  const float* bi = br + (int64_t)h * w;
  const float* f = fval + d.f_off;
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < h && n0 + 32 * (wv & 1) < w;
  auto st = [&](int a, int b, float2 v) {
    if (a < h && b < w) { er[(int64_t)a * w + b] = v.x; ei[(int64_t)a * w + b] = v.y; }
  };
  // rows of B (tall) or V (wide) scaled by f, and rows of V: k-contiguous,
  // fetched eight at a time
  auto scaled_rows = [&](const float* xr, const float* xi, int m, int k0, float2(&v)[8]) {
    const int nv = m < h ? r - k0 : 0;
    float a[8], b[8], s8[8];
    load8(xr + (int64_t)m * n + k0, nv, a);
    load8(xi + (int64_t)m * n + k0, nv, b);
    load8(f + k0, nv, s8);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = make_float2(a[j] * s8[j], b[j] * s8[j]);
  };
  if (d.tall) {
    auto fa = [&](int m, int k0, float2(&v)[8]) { scaled_rows(br, bi, m, k0, v); };
    auto fb = [&](int k0, int c, float2(&v)[8]) {
      const int nv = c < w ? r - k0 : 0;
      float a[8], b[8];
      load8(vr + (int64_t)c * n + k0, nv, a);
      load8(vi + (int64_t)c * n + k0, nv, b);
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = make_float2(a[j], -b[j]);
    };
    mfma_ctile<MODE, true, true, true, true>(m0, n0, r, fa, fb, st, sm, active);
  } else {
    auto fa = [&](int m, int k0, float2(&v)[8]) { scaled_rows(vr, vi, m, k0, v); };
    auto fb = [&](int k, int c) -> float2 {
      if (k >= r || c >= w) return make_float2(0.f, 0.f);
      return make_float2(br[(int64_t)k * w + c], bi[(int64_t)k * w + c]);
    };
    mfma_ctile<MODE, true, false, true, false>(m0, n0, r, fa, fb, st, sm, active);
  }
}

// ------------------------------------------------ t-SVT derivative (JVP) ---
// The t-SVT is the prox of a convex function, so its Jacobian is symmetric
// and the cotangent of the input is the derivative along the output
// cotangent.  With the Gram G = M^H M = V diag(lambda) V^H (tall slice),
// SVT(M) = M g(G), g(lambda) = max(1 - t / sqrt(lambda), 0), and the
// Daleckii-Krein rule for the derivative of a matrix function gives, for a
// direction D with B = M V, C = D V:
//   SVT'(M)[D] = (C diag(g) + B W) V^H,  W = g1 o (C^H B + B^H C),
//   g1_ij = (g_i - g_j) / (lambda_i - lambda_j)   (g' on the diagonal):
//     both sigma > t:  t / (s_i s_j (s_i + s_j));  one above: g / (s^2 - s'^2);
//     none: 0.
// Wide slices use G = M M^H = U diag(lambda) U^H, SVT(M) = g(G) M, with
// B = U^H M, C = U^H D:  SVT'(M)[D] = U (diag(g) C + W B),
// W = g1 o (C B^H + B C^H).  sigma_i = ||B e_i|| (the column or row norm of
// B, taken from M like the forward pass).
// The threshold derivative is dSVT/dt = -B diag(1[s > t] / s) V^H (or
// -U diag(1[s > t] / s) B); its inner product with D is
// -sum_{s_i > t} Re <c_i, b_i> / s_i, weighted by the slice's Fourier weight.

LRSTV_DEV double g1_pair(double si, double sj, double t) {
  const bool ai = si > t, aj = sj > t;
  if (ai && aj) return t / (si * sj * (si + sj));
  if (ai) return (1.0 - t / si) / ((si - sj) * (si + sj));
  if (aj) return (1.0 - t / sj) / ((sj - si) * (sj + si));
  return 0.0;
}

// Per column c of a slice: sigma_c, g_c and the threshold-derivative term
// acon_c = -1[s > t] Re<c_c, b_c> / s * fw / mu  (d/d alpha of <E, D>).
__global__ void __launch_bounds__(256) k_vjp_sigma(const SliceDesc* __restrict__ desc, const float* __restrict__ Bb,
                                                   const float* __restrict__ Cb, float* __restrict__ sig,
                                                   float* __restrict__ gval, double* __restrict__ acon,
                                                   const int* __restrict__ rcount, const double* __restrict__ mu_dev,
                                                   double alpha, float thresh) {
  __shared__ double red[8];
  const SliceDesc d = desc[blockIdx.y];
  const int r = rcount[blockIdx.y], c = blockIdx.x, n = d.n1;
  if (c >= n) return;
  if (c >= r) {  // no eigenpair (zero slice): nothing flows through this column
    if (threadIdx.x == 0) {
      sig[d.f_off + c] = 0.f;
      gval[d.f_off + c] = 0.f;
      acon[d.f_off + c] = 0.0;
    }
    return;
  }
  const int h = d.h, w = d.w;
  const float* br = Bb + d.b_off;
  const float* bi = br + (int64_t)h * w;
  const float* cr = Cb + d.b_off;
  const float* ci = cr + (int64_t)h * w;
  double s2 = 0.0, dt = 0.0;
  if (d.tall) {
    for (int i = threadIdx.x; i < h; i += blockDim.x) {
      const int64_t q = (int64_t)i * n + c;
      const double a = br[q], b = bi[q];
      s2 += a * a + b * b;
      dt += (double)cr[q] * a + (double)ci[q] * b;
    }
  } else {
    for (int i = threadIdx.x; i < w; i += blockDim.x) {
      const int64_t q = (int64_t)c * w + i;
      const double a = br[q], b = bi[q];
      s2 += a * a + b * b;
      dt += (double)cr[q] * a + (double)ci[q] * b;
    }
  }
  s2 = block_sum(s2, red);
  dt = block_sum(dt, red);
  if (threadIdx.x == 0) {
    const double mu = mu_dev ? *mu_dev : 1.0;
    const double t = mu_dev ? alpha / mu : (double)thresh;
    const double sg = sqrt(s2);
    const bool keep = sg > t;
    sig[d.f_off + c] = (float)sg;
    gval[d.f_off + c] = keep ? (float)(1.0 - t / sg) : 0.f;
    acon[d.f_off + c] = keep ? -dt / sg * (double)d.fw / mu : 0.0;
  }
}

// W = g1 o (C^H B + B^H C) (tall) or g1 o (C B^H + B C^H) (wide), r x r,
// as one product over the stacked contraction [C; B] (rows padded to 32).
template <int MODE>
__global__ void __launch_bounds__(256) k_vjp_w(const SliceDesc* __restrict__ desc, const float* __restrict__ Bb,
                                               const float* __restrict__ Cb, const float* __restrict__ sig,
                                               float* __restrict__ Wb, const int* __restrict__ rcount,
                                               const double* __restrict__ mu_dev, double alpha, float thresh) {
  __shared__ MfmaSmem sm;
  const SliceDesc d = desc[blockIdx.z];
  const int r = rcount[blockIdx.z], n = d.n1, h = d.h, w = d.w;
  const int m0 = blockIdx.y * kMT, n0 = blockIdx.x * kMT;
  if (m0 >= r || n0 >= r) return;
  const float* br = Bb + d.b_off;
  const float* bi = br + (int64_t)h * w;
  const float* cr = Cb + d.b_off;
  const float* ci = cr + (int64_t)h * w;
  const float* sg = sig + d.f_off;
  float* wr = Wb + d.v_off;
  float* wi = wr + (int64_t)n * n;
  const double t = mu_dev ? alpha / *mu_dev : (double)thresh;
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < r && n0 + 32 * (wv & 1) < r;
  auto st = [&](int i, int j, float2 v) {
    if (i < r && j < r) {
      const float g = (float)g1_pair(sg[i], sg[j], t);
      wr[(int64_t)i * n + j] = g * v.x;
      wi[(int64_t)i * n + j] = g * v.y;
    }
  };
  if (d.tall) {  // rows k of B, C (ld n), k < h
    const int mp = (h + 31) & ~31;
    auto fa = [&](int i, int k) -> float2 {
      const bool second = k >= mp;
      const int kk = second ? k - mp : k;
      if (i >= r || kk >= h) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)kk * n + i;
      return second ? make_float2(br[q], -bi[q]) : make_float2(cr[q], -ci[q]);
    };
    auto fb = [&](int k, int j) -> float2 {
      const bool second = k >= mp;
      const int kk = second ? k - mp : k;
      if (j >= r || kk >= h) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)kk * n + j;
      return second ? make_float2(cr[q], ci[q]) : make_float2(br[q], bi[q]);
    };
    mfma_ctile<MODE, false, false>(m0, n0, 2 * mp, fa, fb, st, sm, active);
  } else {  // columns k of B, C (rows i < r, ld w), k < w
    const int mp = (w + 31) & ~31;
    auto fa = [&](int i, int k) -> float2 {
      const bool second = k >= mp;
      const int kk = second ? k - mp : k;
      if (i >= r || kk >= w) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)i * w + kk;
      return second ? make_float2(br[q], bi[q]) : make_float2(cr[q], ci[q]);
    };
    auto fb = [&](int k, int j) -> float2 {
      const bool second = k >= mp;
      const int kk = second ? k - mp : k;
      if (j >= r || kk >= w) return make_float2(0.f, 0.f);
      const int64_t q = (int64_t)j * w + kk;
      return second ? make_float2(cr[q], -ci[q]) : make_float2(br[q], -bi[q]);
    };
    mfma_ctile<MODE, true, true>(m0, n0, 2 * mp, fa, fb, st, sm, active);
  }
}

// tall: R (h x r, ld n) = B W + C diag(g);  wide: R (r x w, ld w) = W B + diag(g) C
template <int MODE>
__global__ void __launch_bounds__(256) k_vjp_r(const SliceDesc* __restrict__ desc, const float* __restrict__ Bb,
                                               const float* __restrict__ Cb, const float* __restrict__ Wb,
                                               const float* __restrict__ gval, float* __restrict__ Rb,
                                               const int* __restrict__ rcount) {
  __shared__ MfmaSmem sm;
  const SliceDesc d = desc[blockIdx.z];
  const int r = rcount[blockIdx.z], n = d.n1, h = d.h, w = d.w;
  const int M = d.tall ? h : r, N = d.tall ? r : w, ld = d.tall ? n : w;
  const int m0 = blockIdx.y * kMT, n0 = blockIdx.x * kMT;
  if (m0 >= M || n0 >= N) return;
  const float* br = Bb + d.b_off;
  const float* bi = br + (int64_t)h * w;
  const float* cr = Cb + d.b_off;
  const float* ci = cr + (int64_t)h * w;
  const float* wr = Wb + d.v_off;
  const float* wi = wr + (int64_t)n * n;
  const float* g = gval + d.f_off;
  float* rr = Rb + d.b_off;
  float* ri = rr + (int64_t)h * w;
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < M && n0 + 32 * (wv & 1) < N;
  const bool tall = d.tall;
  auto st = [&](int a, int b, float2 v) {
    if (a < M && b < N) {
      const int64_t q = (int64_t)a * ld + b;
      const float s = tall ? g[b] : g[a];
      rr[q] = v.x + s * cr[q];
      ri[q] = v.y + s * ci[q];
    }
  };
  if (tall) {
    auto fa = [&](int i, int k) -> float2 {
      if (i >= h || k >= r) return make_float2(0.f, 0.f);
      return make_float2(br[(int64_t)i * n + k], bi[(int64_t)i * n + k]);
    };
    auto fb = [&](int k, int j) -> float2 {
      if (k >= r || j >= r) return make_float2(0.f, 0.f);
      return make_float2(wr[(int64_t)k * n + j], wi[(int64_t)k * n + j]);
    };
    mfma_ctile<MODE, true, false>(m0, n0, r, fa, fb, st, sm, active);
  } else {
    auto fa = [&](int i, int k) -> float2 {
      if (i >= r || k >= r) return make_float2(0.f, 0.f);
      return make_float2(wr[(int64_t)i * n + k], wi[(int64_t)i * n + k]);
    };
    auto fb = [&](int k, int j) -> float2 {
      if (k >= r || j >= w) return make_float2(0.f, 0.f);
      return make_float2(br[(int64_t)k * w + j], bi[(int64_t)k * w + j]);
    };
    mfma_ctile<MODE, true, false>(m0, n0, r, fa, fb, st, sm, active);
  }
}

// ------------------------------------------------------------ launcher ---
// Tridiagonalisation shapes, chosen per handle by the autotuner.  Shape code
// 100 kind + waves: kind 0 is k_tridiag_reg (rows in VGPRs and LDS; more
// waves hide the LDS and cross-lane latency of the per-row reductions, the
// rows per wave keep the LDS part of the packed Gram under 160 KB), kind 1
// is k_tridiag_mfma (32 x 32 register tiles, rank-2 update on the matrix
// cores; static LDS, slices up to 256).
struct TriShape {
  int kind, nw, jr;
};
static const TriShape kTriShapes[kTriVariants] = {{0, 8, 10}, {0, 12, 7}, {0, 16, 6}, {1, 12, 3}, {1, 8, 5}};
// Dynamic LDS granted per row variant (host-side function attribute, set
// outside any stream capture by prepare_svt), and the device's LDS per block.
static size_t g_tri_granted[kTriVariants] = {65536, 65536, 65536, 0, 0};
static int g_lds_max = 65536;

int tri_variant_code(int v) { return 100 * kTriShapes[v].kind + kTriShapes[v].nw; }

// Dynamic LDS of k_tridiag_reg: the packed LDS rows plus (3 + NW) n complex
// (two columns, w, NW column-part rows).
static size_t tridiag_reg_lds(int n, int v) {
  const int NW = kTriShapes[v].nw, JR = kTriShapes[v].jr;
  const int RL = n > NW * JR ? n - NW * JR : 0;
  return ((size_t)RL * (RL + 1) / 2 + (size_t)(3 + NW) * n) * sizeof(float2);
}
// Static LDS of k_tridiag_mfma<NW, TPW>: seven columns (x and a per step
// parity, the column after them, v, w) and NW partial rows (256 complex
// each).
static size_t tridiag_mfma_lds(int nw) { return (size_t)(7 + nw) * 256 * sizeof(float2) + 1024; }

static const void* tri_kernel(int v) {
  switch (v) {
    case 0: return (const void*)k_tridiag_reg<10, 8>;
    case 1: return (const void*)k_tridiag_reg<7, 12>;
    case 2: return (const void*)k_tridiag_reg<6, 16>;
    case 3: return (const void*)k_tridiag_mfma<12, 3>;
    default: return (const void*)k_tridiag_mfma<8, 5>;
  }
}

bool tri_variant_onchip(int v, int n) {
  if (n > 256) return false;
  if (kTriShapes[v].kind == 1) return (int)tridiag_mfma_lds(kTriShapes[v].nw) <= g_lds_max;
  return tridiag_reg_lds(n, v) <= g_tri_granted[v];
}

// With the register-tile kernels, slices with n <= kTriSmallN and larger
// ones are reduced by two launches (a 4-wave shape of which three blocks fit a
// CU, and the tuned shape of one block per CU).
static bool tridiag_two_classes(const SvtLaunch& L) {
  const int v = (L.tri_variant >= 0 && L.tri_variant < kTriVariants) ? L.tri_variant : kTriDefault;
  return v >= 3 && tri_variant_onchip(v, L.max_n1) && L.min_n1 <= kTriSmallN && L.max_n1 > kTriSmallN;
}

// which: bit 0 the slices with n <= kTriSmallN, bit 1 the larger ones (the
// register-tile kernels; other shapes take every slice either way).
void launch_svt_tridiag(const SvtLaunch& L, hipStream_t s, int which) {
  const int n = L.max_n1, ns = L.n_slices;
  const int v = (L.tri_variant >= 0 && L.tri_variant < kTriVariants) ? L.tri_variant : kTriDefault;
  if (tri_variant_onchip(v, n)) {
    const size_t lds = kTriShapes[v].kind == 0 ? tridiag_reg_lds(n, v) : 0;
    switch (v) {
      case 0: hipLaunchKernelGGL((k_tridiag_reg<10, 8>), dim3(ns), dim3(512), lds, s, L.desc, L.gram, L.tri, L.halt); break;
      case 1: hipLaunchKernelGGL((k_tridiag_reg<7, 12>), dim3(ns), dim3(768), lds, s, L.desc, L.gram, L.tri, L.halt); break;
      case 2: hipLaunchKernelGGL((k_tridiag_reg<6, 16>), dim3(ns), dim3(1024), lds, s, L.desc, L.gram, L.tri, L.halt); break;
      default: {
        // Slices with n <= 128 take a 4-wave block (three per CU: their
        // per-step latencies overlap), the others the tuned shape.
        const bool small = L.min_n1 <= kTriSmallN;
        if (small && (which & 1))
          hipLaunchKernelGGL((k_tridiag_mfma<4, 3, kTriSmallN>), dim3(ns), dim3(256), 0, s, L.desc, L.gram, L.tri,
                             L.halt, 0);
        if (n <= kTriSmallN || !(which & 2)) break;
        const int nmin = small ? kTriSmallN : 0;
        if (v == 3)
          hipLaunchKernelGGL((k_tridiag_mfma<12, 3>), dim3(ns), dim3(768), 0, s, L.desc, L.gram, L.tri, L.halt, nmin);
        else
          hipLaunchKernelGGL((k_tridiag_mfma<8, 5>), dim3(ns), dim3(512), 0, s, L.desc, L.gram, L.tri, L.halt, nmin);
        break;
      }
    }
  } else {
    hipLaunchKernelGGL(k_tridiag<false>, dim3(ns), dim3(256), (size_t)(2 + 4) * n * sizeof(float2), s, L.desc,
                       L.gram, L.tri, L.halt);
  }
}
static void launch_tridiag(const SvtLaunch& L, hipStream_t s) { launch_svt_tridiag(L, s, 3); }

static void launch_gram_bf16(const SvtLaunch& L, hipStream_t s) {
  const int ns = L.n_slices, T2 = (L.max_n1 + 127) / 128;
  hipLaunchKernelGGL(k_gram_bf16, dim3(xcd_grid(T2 * (T2 + 1) / 2, ns)), dim3(256), 0, s, L.desc, L.slices, L.gram,
                     T2 * (T2 + 1) / 2, ns, L.halt);
}

void launch_svt_gram(const SvtLaunch& L, hipStream_t s) {
  const int ns = L.n_slices, n = L.max_n1;
  const int TT = (n + kMT - 1) / kMT;
  if (L.precision == LRSTV_SPLIT_BF16)
    launch_gram_bf16(L, s);
  else
    hipLaunchKernelGGL(k_gram<kF32>, dim3(xcd_grid(TT * (TT + 1) / 2, ns)), dim3(256), 0, s, L.desc, L.slices, L.gram,
                       TT * (TT + 1) / 2, ns, L.halt);
}

void prepare_svt(int max_n1) {
  const int n = max_n1;
  if (n > 256) return;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    g_lds_max = (int)prop.sharedMemPerBlock;
  for (int v = 0; v < kTriVariants; ++v) {
    if (kTriShapes[v].kind != 0) continue;
    const size_t need = tridiag_reg_lds(n, v);
    if (need <= g_tri_granted[v] || (int)need + 2048 > g_lds_max) continue;
    if (hipFuncSetAttribute(tri_kernel(v), hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) == hipSuccess)
      g_tri_granted[v] = need;
    else
      (void)hipGetLastError();  // clear the sticky error: the global-memory variant is used instead
  }
}
static void launch_trivec(const SvtLaunch& L, hipStream_t s, size_t eig_lds, const double* mu, float thresh) {
  const int ns = L.n_slices, n = L.max_n1;
  constexpr int VB = 64;
  hipLaunchKernelGGL(k_trieig<1>, dim3((n + VB - 1) / VB, ns), dim3(VB), eig_lds, s, L.desc, L.tri, L.xs, L.V,
                     L.rcount, mu, L.alpha, thresh, 0, L.halt);
  hipLaunchKernelGGL(k_trieig<2>, dim3(ns), dim3(1024), eig_lds, s, L.desc, L.tri, L.xs, L.V, L.rcount, mu, L.alpha,
                     thresh, 0, L.halt);
}

static size_t tridiag_onchip_bytes(int n) {
  return ((size_t)n * (n + 1) / 2 + 2 * (size_t)n + 4 * (size_t)n) * sizeof(float2);
}

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

// Every stage after the tridiagonalisation, on one stream.
static void svt_after_tridiag(const SvtLaunch& L, hipStream_t s, StageTimer& T) {
  const int ns = L.n_slices, n = L.max_n1, m = L.max_m1;
  const bool bf = L.precision == LRSTV_SPLIT_BF16;
  const int TM = (m + kMT - 1) / kMT;
  const size_t eig_lds = (size_t)5 * n * sizeof(double) + (size_t)(n + 1 + 1024) * sizeof(int);
  T.begin(ST_TRIEIG);
  const int probes = eig_probes(ns, n), epb = 256 / probes;
  hipLaunchKernelGGL(k_trieig<0>, dim3((n + epb - 1) / epb, ns), dim3(256), eig_lds, s, L.desc, L.tri, L.xs, L.V,
                     L.rcount, L.mu, L.alpha, L.thresh, probes, L.halt);
  T.end(ST_TRIEIG);
  T.begin(ST_TRIVEC);
  launch_trivec(L, s, eig_lds, L.mu, L.thresh);
  T.end(ST_TRIVEC);
  T.begin(ST_BACKTRANS);
  launch_backtrans(L, s);
  T.end(ST_BACKTRANS);
  // B: tall h x r, wide r x w -> tiles over (max(n, m)) both ways
  T.begin(ST_BP1);
  if (bf)
    hipLaunchKernelGGL(k_bp1<kBF16x3>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, L.slices, L.V, L.B,
                       L.rcount, TM, ns, L.halt);
  else
    hipLaunchKernelGGL(k_bp1<kF32>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, L.slices, L.V, L.B, L.rcount,
                       TM, ns, L.halt);
  T.end(ST_BP1);
  T.begin(ST_COLNORM);
  hipLaunchKernelGGL(k_colnorm, dim3((n + 63) / 64, ns), dim3(256), 0, s, L.desc, L.B, L.fval, L.rcount, L.mu, L.alpha,
                     L.thresh, L.halt);
  T.end(ST_COLNORM);
  T.begin(ST_BP2);
  if (bf)
    hipLaunchKernelGGL(k_bp2<kBF16x3>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, L.slices, L.V, L.B,
                       L.fval, L.rcount, TM, ns, L.halt);
  else
    hipLaunchKernelGGL(k_bp2<kF32>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, L.slices, L.V, L.B,
                       L.fval, L.rcount, TM, ns, L.halt);
  T.end(ST_BP2);
}

int svt_split_point(int n_slices) {
  const int cus = device_cus();
  if (n_slices <= cus || n_slices % cus == 0) return 0;
  return n_slices - n_slices % cus;
}

void launch_svt(const SvtLaunch& L, hipStream_t s, StageTimer* tm, const SvtSplit* sp) {
  StageTimer dummy;
  StageTimer& T = tm ? *tm : dummy;
  const int ns = L.n_slices, n = L.max_n1;
  if (ns == 0) return;
  const bool bf = L.precision == LRSTV_SPLIT_BF16;
  const int TT = (n + kMT - 1) / kMT;
  T.begin(ST_GRAM);
  if (bf)
    launch_gram_bf16(L, s);
  else
    hipLaunchKernelGGL(k_gram<kF32>, dim3(xcd_grid(TT * (TT + 1) / 2, ns)), dim3(256), 0, s, L.desc, L.slices, L.gram,
                       TT * (TT + 1) / 2, ns, L.halt);
  T.end(ST_GRAM);
  // per-stage timing keeps one stream (every stage times all the slices)
  if (sp && sp->s2 && sp->first > 0 && sp->first < ns && !T.on) {
    SvtLaunch A = L, B = L;
    A.n_slices = sp->first;
    B.desc = L.desc + sp->first;
    B.rcount = L.rcount + sp->first;
    B.n_slices = ns - sp->first;
    if (sp->big && tridiag_two_classes(A)) {
      // the first group's slices above kTriSmallN (one block per CU) on the
      // second stream beside its smaller ones (three per CU), so that the
      // last round of either launch finds the other's blocks to run; the
      // second group follows them there
      (void)hipEventRecord(sp->fork, s);
      (void)hipStreamWaitEvent(sp->s2, sp->fork, 0);
      launch_svt_tridiag(A, sp->s2, 2);
      launch_svt_tridiag(A, s, 1);
      (void)hipEventRecord(sp->big, sp->s2);
      (void)hipStreamWaitEvent(s, sp->big, 0);
    } else {
      launch_tridiag(A, s);
      (void)hipEventRecord(sp->fork, s);
      (void)hipStreamWaitEvent(sp->s2, sp->fork, 0);
    }
    // the second group's tridiagonalisation is queued before the first
    // group's next stage, so that its blocks are placed first
    launch_tridiag(B, sp->s2);
    svt_after_tridiag(A, s, T);
    svt_after_tridiag(B, sp->s2, T);
    (void)hipEventRecord(sp->join, sp->s2);
    (void)hipStreamWaitEvent(s, sp->join, 0);
    return;
  }
  T.begin(ST_TRIDIAG);
  launch_tridiag(L, s);
  T.end(ST_TRIDIAG);
  svt_after_tridiag(L, s, T);
}


void launch_sym_eig(const SvtLaunch& L, hipStream_t s) {
  const int ns = L.n_slices, n = L.max_n1;
  if (ns == 0) return;
  launch_tridiag(L, s);
  const size_t eig_lds = (size_t)5 * n * sizeof(double) + (size_t)(n + 1 + 1024) * sizeof(int);
  const int probes = eig_probes(ns, n), epb = 256 / probes;
  hipLaunchKernelGGL(k_trieig<0>, dim3((n + epb - 1) / epb, ns), dim3(256), eig_lds, s, L.desc, L.tri, L.xs, L.V,
                     L.rcount, (const double*)nullptr, 0.0, -1.f, probes, L.halt);
  launch_trivec(L, s, eig_lds, nullptr, -1.f);
  launch_backtrans(L, s);
}

void launch_svt_vjp(const SvtVjpLaunch& J, hipStream_t s) {
  const SvtLaunch& L = J.fw;
  const int ns = L.n_slices, n = L.max_n1, m = L.max_m1;
  if (ns == 0) return;
  const int TT = (n + kMT - 1) / kMT, TM = (m + kMT - 1) / kMT;
  // full eigendecomposition of every Gram (thresh < 0: all eigenpairs)
  hipLaunchKernelGGL(k_gram<kF32>, dim3(xcd_grid(TT * (TT + 1) / 2, ns)), dim3(256), 0, s, L.desc, L.slices, L.gram,
                       TT * (TT + 1) / 2, ns, L.halt);
  launch_tridiag(L, s);
  const size_t eig_lds = (size_t)5 * n * sizeof(double) + (size_t)(n + 1 + 1024) * sizeof(int);
  const int probes = eig_probes(ns, n), epb = 256 / probes;
  hipLaunchKernelGGL(k_trieig<0>, dim3((n + epb - 1) / epb, ns), dim3(256), eig_lds, s, L.desc, L.tri, L.xs, L.V,
                     L.rcount, (const double*)nullptr, 0.0, -1.f, probes, L.halt);
  launch_trivec(L, s, eig_lds, nullptr, -1.f);
  launch_backtrans(L, s);
  // B = M V, C = D V (or U^H M, U^H D)
  hipLaunchKernelGGL(k_bp1<kF32>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, L.slices, L.V, L.B, L.rcount,
                       TM, ns, L.halt);
  hipLaunchKernelGGL(k_bp1<kF32>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, J.dsl, L.V, J.C, L.rcount, TM,
                     ns, L.halt);
  hipLaunchKernelGGL(k_vjp_sigma, dim3(n, ns), dim3(256), 0, s, L.desc, L.B, J.C, J.sig, L.fval, J.acon, L.rcount,
                     L.mu, L.alpha, L.thresh);
  hipLaunchKernelGGL(k_vjp_w<kF32>, dim3(TT, TT, ns), dim3(256), 0, s, L.desc, L.B, J.C, J.sig, J.W, L.rcount,
                     L.mu, L.alpha, L.thresh);
  hipLaunchKernelGGL(k_vjp_r<kF32>, dim3(TM, TM, ns), dim3(256), 0, s, L.desc, L.B, J.C, J.W, L.fval, J.R,
                     L.rcount);
  // result (R V^H or U R) over the direction slices
  hipLaunchKernelGGL(k_bp2<kF32>, dim3(xcd_grid(TM * TM, ns)), dim3(256), 0, s, L.desc, J.dsl, L.V, J.R, J.ones,
                     L.rcount, TM, ns, L.halt);
}

}  // namespace lrstv
