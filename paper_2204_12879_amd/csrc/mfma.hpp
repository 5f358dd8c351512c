// Complex GEMM tile on the CDNA4 matrix cores.
//
// A 256-thread block (4 waves) computes a 64 x 64 complex tile
// C = sum_k A(m, k) B(k, n); wave q owns the 32 x 32 sub-tile
// (32 (q >> 1), 32 (q & 1)).  Operands are fetched through accessors
// fa(m, k), fb(k, n) that return float2 (zero outside the matrix), staged
// through LDS in chunks of 32 along k with a register prefetch of the next
// chunk.
//
// Two arithmetic modes:
//   kF32   v_mfma_f32_32x32x2f32: FP32 operands, FP32 accumulation, three
//          real products per complex one (the 3M method: P1 = Re A Re B,
//          P2 = Im A Im B, P3 = (Re A + Im A)(Re B + Im B); Re C = P1 - P2,
//          Im C = P3 - P1 - P2), the sums formed as the operands are read.
//          On CDNA4 the FP32 matrix instructions run at the packed-FP32
//          vector rate and occupy the same pipeline, so a product saved is
//          time saved.
//   kBF16x3 split-BF16: every FP32 operand x is stored as hi = bf16(x),
//          lo = bf16(x - hi); a real product is hi*hi + hi*lo + lo*hi
//          (the lo*lo term, ~2^-16 relative, is dropped), each term a
//          v_mfma_f32_32x32x16_bf16 with FP32 accumulation, four real
//          products per complex one
//            Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B.
//
// Lane layouts (checked on gfx950): for both instructions lane l holds
// A(l % 32, k) and B(k, l % 32) with k = l / 32 (f32, K = 2) or
// k = 8 (l / 32) + e, e = 0..7 (bf16, K = 16); accumulator element r of
// lane l is C(8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
#pragma once
#include "common.hpp"

namespace lrstv {

typedef float f32x16 __attribute__((ext_vector_type(16)));
// v_mfma_f32_16x16x4f32: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16);
// accumulator element r of lane l is C(4 (l / 16) + r, l % 16).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum MfmaMode { kF32 = 0, kBF16x3 = 1 };

constexpr int kMT = 64;   // block tile (rows and columns)
constexpr int kKC = 32;   // k chunk staged per pass
constexpr int kBfPad = 8; // bf16 row padding (keeps 16-byte alignment)

struct MfmaSmemF32 {
  float ar[kKC][kMT + 1], ai[kKC][kMT + 1], br[kKC][kMT + 1], bi[kKC][kMT + 1];
};
struct MfmaSmemBF {
  // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo; rows are m (A) or n (B),
  // k contiguous so a lane's 8 consecutive k are one 16-byte read
  __bf16 a[4][kMT][kKC + kBfPad];
  __bf16 b[4][kMT][kKC + kBfPad];
};
union MfmaSmem {
  MfmaSmemF32 f;
  MfmaSmemBF h;
};

// kF32: re, im, p3 accumulate P1, P2, P3 of the 3M method (combined by
// cacc_result); kBF16x3: re and im are the result and p3 is unused.
struct CAcc {
  f32x16 re, im, p3;
};
template <int MODE, bool M3>
LRSTV_DEV float2 cacc_result(const CAcc& c, int r) {
  if (MODE == kF32 && M3) return make_float2(c.re[r] - c.im[r], c.p3[r] - c.re[r] - c.im[r]);
  return make_float2(c.re[r], c.im[r]);
}

LRSTV_DEV bf16x8 bf_neg(bf16x8 x) {
  union {
    bf16x8 v;
    uint32_t u[4];
  } t;
  t.v = x;
#pragma unroll
  for (int i = 0; i < 4; ++i) t.u[i] ^= 0x80008000u;
  return t.v;
}

// Thread t stages 8 consecutive k of one row (m for A, n for B).  When k is
// the contiguous memory index (KFAST) a row's 32 k are split over 4 lanes;
// otherwise lanes run along the row index so each load is coalesced.
template <bool KFAST>
LRSTV_DEV void stage_coords(int t, int& row, int& k0) {
  if (KFAST) {
    row = t >> 2;
    k0 = 8 * (t & 3);
  } else {
    row = t & 63;
    k0 = 8 * (t >> 6);
  }
}

template <int MODE>
LRSTV_DEV void stage_store(MfmaSmem& sm, bool isA, int row, int k0, const float2 (&v)[8]) {
  if (MODE == kF32) {
    float(*pr)[kMT + 1] = isA ? sm.f.ar : sm.f.br;
    float(*pi)[kMT + 1] = isA ? sm.f.ai : sm.f.bi;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      pr[k0 + j][row] = v[j].x;
      pi[k0 + j][row] = v[j].y;
    }
  } else {
    bf16x8 rh, rl, ih, il;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const __bf16 a = (__bf16)v[j].x, b = (__bf16)v[j].y;
      rh[j] = a;
      rl[j] = (__bf16)(v[j].x - (float)a);
      ih[j] = b;
      il[j] = (__bf16)(v[j].y - (float)b);
    }
    __bf16(*p)[kMT][kKC + kBfPad] = isA ? sm.h.a : sm.h.b;
    *(bf16x8*)&p[0][row][k0] = rh;
    *(bf16x8*)&p[1][row][k0] = rl;
    *(bf16x8*)&p[2][row][k0] = ih;
    *(bf16x8*)&p[3][row][k0] = il;
  }
}

template <int MODE, bool M3>
LRSTV_DEV void chunk_mma(const MfmaSmem& sm, int wy, int wx, int lane, bool active, CAcc& c) {
  if (!active) return;
  const int li = lane & 31, lk = lane >> 5;
  if (MODE == kF32) {
#pragma unroll 4
    for (int kk = 0; kk < kKC / 2; ++kk) {
      const int k = 2 * kk + lk;
      const float ar = sm.f.ar[k][32 * wy + li], ai = sm.f.ai[k][32 * wy + li];
      const float br = sm.f.br[k][32 * wx + li], bi = sm.f.bi[k][32 * wx + li];
      if (M3) {
        c.re = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, c.re, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, c.im, 0, 0, 0);
        c.p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar + ai, br + bi, c.p3, 0, 0, 0);
      } else {
        c.re = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, c.re, 0, 0, 0);
        c.re = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, c.re, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, c.im, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, c.im, 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < kKC / 16; ++ks) {
      const int ko = 16 * ks + 8 * lk;
      const int ra = 32 * wy + li, rb = 32 * wx + li;
      const bf16x8 arh = *(const bf16x8*)&sm.h.a[0][ra][ko], arl = *(const bf16x8*)&sm.h.a[1][ra][ko];
      const bf16x8 aih = *(const bf16x8*)&sm.h.a[2][ra][ko], ail = *(const bf16x8*)&sm.h.a[3][ra][ko];
      const bf16x8 brh = *(const bf16x8*)&sm.h.b[0][rb][ko], brl = *(const bf16x8*)&sm.h.b[1][rb][ko];
      const bf16x8 bih = *(const bf16x8*)&sm.h.b[2][rb][ko], bil = *(const bf16x8*)&sm.h.b[3][rb][ko];
      const bf16x8 naih = bf_neg(aih), nail = bf_neg(ail);
      // small terms first, then the hi*hi term
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, c.re, 0, 0, 0);
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, c.re, 0, 0, 0);
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih, bil, c.re, 0, 0, 0);
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nail, bih, c.re, 0, 0, 0);
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, c.re, 0, 0, 0);
      c.re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih, bih, c.re, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bil, c.im, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bih, c.im, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brl, c.im, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, brh, c.im, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bih, c.im, 0, 0, 0);
      c.im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brh, c.im, 0, 0, 0);
    }
  }
}

// Eight consecutive floats p[0 .. 7], of which the first nvalid exist (the
// rest read as 0): two float4 loads when all eight exist and p is 16-byte
// aligned, element loads otherwise.
LRSTV_DEV void load8(const float* p, int nvalid, float (&v)[8]) {
  if (nvalid >= 8 && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < nvalid ? p[j] : 0.f;
  }
}

// Four consecutive floats p[0 .. 3], of which the first nvalid exist: one
// float4 load when all four exist and p is 16-byte aligned.
LRSTV_DEV void load4(const float* p, int nvalid, float (&v)[4]) {
  if (nvalid >= 4 && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = j < nvalid ? p[j] : 0.f;
  }
}

// C(m0 .. m0+63, n0 .. n0+63) = sum_{k < K} fa(m, k) fb(k, n).
// AK / BK: k is the contiguous memory index of A / B (selects the staging
// order).  With VA / VB the accessor is wide instead: for a k-contiguous
// operand eight-wide along k, fa(m, k, v) / fb(k, n, v) filling v[j] with the
// values at k + j (see load8); for the other operands (FP32 mode only)
// four-wide along the row / column index, fa(m, k, v) / fb(k, n, v) filling
// v[j] with the values at m + j / n + j (see load4), a thread staging four
// consecutive rows (columns) of two k.  `active` (wave-uniform) skips the
// products of a wave whose sub-tile is not needed; every wave still takes
// part in staging.  The result is handed to st(row, col, float2) for rows and
// columns of the wave's sub-tile.
template <int MODE, bool AK, bool BK, bool VA = false, bool VB = false, bool M3 = true, class FA, class FB, class ST>
LRSTV_DEV void mfma_ctile(int m0, int n0, int K, FA fa, FB fb, ST st, MfmaSmem& sm, bool active) {
  constexpr bool A4 = VA && !AK, B4 = VB && !BK;   // four-wide along the row / column index
  static_assert(MODE == kF32 || !(A4 || B4), "four-wide staging is for the FP32 layout");
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wy = wv >> 1, wx = wv & 1;
  int ra, ka, rb, kb;
  stage_coords<AK>(t, ra, ka);
  stage_coords<BK>(t, rb, kb);
  if constexpr (A4) {
    ra = 4 * (t & 15);
    ka = t >> 4;   // rows ka and ka + 16 of the chunk
  }
  if constexpr (B4) {
    rb = 4 * (t & 15);
    kb = t >> 4;
  }
  CAcc c;
#pragma unroll
  for (int i = 0; i < 16; ++i) c.re[i] = c.im[i] = c.p3[i] = 0.f;
  float2 va[8], vb[8];
  auto fetch = [&](int kc) {
    if constexpr (A4) {
#pragma unroll
      for (int e = 0; e < 2; ++e) fa(m0 + ra, kc + ka + 16 * e, *reinterpret_cast<float2(*)[4]>(&va[4 * e]));
    } else if constexpr (VA) {
      fa(m0 + ra, kc + ka, va);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) va[j] = fa(m0 + ra, kc + ka + j);
    }
    if constexpr (B4) {
#pragma unroll
      for (int e = 0; e < 2; ++e) fb(kc + kb + 16 * e, n0 + rb, *reinterpret_cast<float2(*)[4]>(&vb[4 * e]));
    } else if constexpr (VB) {
      fb(kc + kb, n0 + rb, vb);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) vb[j] = fb(kc + kb + j, n0 + rb);
    }
  };
  // four-wide staging: element (row r + j, k + 16 e) of the chunk
  auto store4 = [&](float (*pr)[kMT + 1], float (*pi)[kMT + 1], int r, int k, const float2 (&v)[8]) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        pr[k + 16 * e][r + j] = v[4 * e + j].x;
        pi[k + 16 * e][r + j] = v[4 * e + j].y;
      }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += kKC) {
    if constexpr (A4) store4(sm.f.ar, sm.f.ai, ra, ka, va);
    else stage_store<MODE>(sm, true, ra, ka, va);
    if constexpr (B4) store4(sm.f.br, sm.f.bi, rb, kb, vb);
    else stage_store<MODE>(sm, false, rb, kb, vb);
    __syncthreads();
    if (k0 + kKC < K) fetch(k0 + kKC);
    chunk_mma<MODE, M3>(sm, wy, wx, lane, active, c);
    __syncthreads();
  }
  if (!active) return;
  const int col = n0 + 32 * wx + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 32 * wy + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    st(row, col, cacc_result<MODE, M3>(c, r));
  }
}

// ----------------------------------------------------------- real tile ---
// Real FP32 GEMM tile on v_mfma_f32_32x32x2f32: C(m0.., n0..) = sum_k
// fa(m, k) fb(k, n), same block shape, staging and lane layouts as the
// complex tile above.
struct MfmaSmemR {
  float a[kKC][kMT + 1], b[kKC][kMT + 1];
};

// t: the thread's index within its group of 256 (a block may run several
// groups on separate tiles; every group calls this the same number of times
// with the same K, since the routine synchronises the whole block).
// With B4, B (not k-contiguous) is fetched four-wide along n: fb(k, n, v)
// fills v[j] with the values at n + j, a thread staging four columns of two k.
template <bool AK, bool BK, bool B4 = false, class FA, class FB, class ST>
LRSTV_DEV void mfma_rtile_t(int t, int m0, int n0, int K, FA fa, FB fb, ST st, MfmaSmemR& sm, bool active) {
  static_assert(!(B4 && BK), "four-wide B staging is for an n-contiguous B");
  const int lane = t & 63, wv = t >> 6, wy = wv >> 1, wx = wv & 1;
  const int li = lane & 31, lk = lane >> 5;
  int ra, ka, rb, kb;
  stage_coords<AK>(t, ra, ka);
  stage_coords<BK>(t, rb, kb);
  if constexpr (B4) {
    rb = 4 * (t & 15);
    kb = t >> 4;   // rows kb and kb + 16 of the chunk
  }
  f32x16 c;
#pragma unroll
  for (int i = 0; i < 16; ++i) c[i] = 0.f;
  float va[8], vb[8];
  auto fetch_b = [&](int kc) {
    if constexpr (B4) {
#pragma unroll
      for (int e = 0; e < 2; ++e) fb(kc + kb + 16 * e, n0 + rb, *reinterpret_cast<float(*)[4]>(&vb[4 * e]));
    } else {
      fb(kc + kb, n0 + rb, vb);
    }
  };
  fa(m0 + ra, ka, va);
  fetch_b(0);
  for (int k0 = 0; k0 < K; k0 += kKC) {
#pragma unroll
    for (int j = 0; j < 8; ++j) sm.a[ka + j][ra] = va[j];
    if constexpr (B4) {
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j) sm.b[kb + 16 * e][rb + j] = vb[4 * e + j];
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) sm.b[kb + j][rb] = vb[j];
    }
    __syncthreads();
    if (k0 + kKC < K) {
      fa(m0 + ra, k0 + kKC + ka, va);
      fetch_b(k0 + kKC);
    }
    if (active) {
#pragma unroll 4
      for (int kk = 0; kk < kKC / 2; ++kk) {
        const int k = 2 * kk + lk;
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(sm.a[k][32 * wy + li], sm.b[k][32 * wx + li], c, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (!active) return;
  const int col = n0 + 32 * wx + li;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 32 * wy + 8 * (r >> 2) + 4 * lk + (r & 3);
    st(row, col, c[r]);
  }
}
template <bool AK, bool BK, class FA, class FB, class ST>
LRSTV_DEV void mfma_rtile(int m0, int n0, int K, FA fa, FB fb, ST st, MfmaSmemR& sm, bool active) {
  mfma_rtile_t<AK, BK>(threadIdx.x, m0, n0, K, fa, fb, st, sm, active);
}

}  // namespace lrstv
