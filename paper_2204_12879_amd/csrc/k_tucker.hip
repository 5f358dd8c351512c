// Truncated-Tucker L-update (Sec. III-C, 1st step, eq. X_solution): the
// average X = 1/2 (O - S - N + Z + (Gamma1 - Gamma2)/mu) is replaced by its
// HOOI approximation of Tucker ranks (r1, r2, r3):
//   start   P_n = projector onto the leading r_n eigenvectors of the mode-n
//           Gram X_(n) X_(n)^T (truncated HOSVD);
//   sweeps  for n = 1, 2, 3: P_n from the Gram of (X x_{m != n} P_m)_(n)
//           (the latest projectors of the other modes);
//   result  L = X x_1 P_1 x_2 P_2 x_3 P_3.
// Projectors P = U U^T (U orthonormal, n x r) replace the factors: the Gram
// of X x_m P_m equals that of X x_m U_m^T, and L is the same.
//
// Kernels (all batched over the cubes of a handle, block ranges per cube
// from a prefix table, FP32 operands on the matrix cores):
//   k_tk_gram<M>    split-K partial Grams of the mode-M unfolding, one
//                   block per (lower 64 x 64 tile, contraction group);
//   k_tk_reduce     fixed-order sum of the partials into the packed lower
//                   complex Gram (imaginary part 0) that the Hermitian
//                   tridiagonalisation reads;
//   k_tk_proj       P = V_r V_r^H (real part) from the eigenvectors;
//   k_tk_prod<M>    Y = X x_M P; the last product of the L-update writes L
//                   and moves T_z = mu L + ... by mu (L_new - L_old).
// Cube layout [b][h][w]; modes 0 (height, axis h), 1 (width, w), 2 (bands).
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace lrstv {

LRSTV_DEV int tk_cube(const int* __restrict__ bstart, int nc, int blk) { return find_cube(bstart, nc, blk); }

// Row index of packed lower entry e (e = r (r + 1) / 2 + c, c <= r).
LRSTV_DEV int packed_row(int64_t e) {
  int r = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
  while ((int64_t)r * (r + 1) / 2 > e) --r;
  while ((int64_t)(r + 1) * (r + 2) / 2 <= e) ++r;
  return r;
}

// ------------------------------------------------------------ mode Grams ---
// Mode M contraction space (per cube): M = 0: (j, x), k = j w + x;
// M = 1: (j, i), k = j h + i; M = 2: p = i w + x.  Group g covers
// k in [g KG, min((g + 1) KG, K)); KG is a multiple of 32.
template <int M>
LRSTV_DEV void tk_gram_fetch(const float* __restrict__ X, const TkGeo& g, int row, int64_t kk, int64_t kend,
                             float (&v)[8]) {
  const int h = g.h, w = g.w, b = g.b;
  const int64_t hw = (int64_t)h * w;
  const int d = M == 0 ? h : (M == 1 ? w : b);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = 0.f;
  if (row >= d || kk >= kend) return;
  const int nval = (int)((kend - kk) < 8 ? (kend - kk) : 8);
  if (M == 0) {
    const int64_t j = kk / w;
    const int x = (int)(kk - j * w);
    if (x + nval <= w) {
      load8(X + j * hw + (int64_t)row * w + x, nval, v);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (e >= nval) break;
        const int64_t k2 = kk + e, j2 = k2 / w;
        v[e] = X[j2 * hw + (int64_t)row * w + (k2 - j2 * w)];
      }
    }
  } else if (M == 1) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (e >= nval) break;
      const int64_t k2 = kk + e, j2 = k2 / h;
      v[e] = X[j2 * hw + (k2 - j2 * h) * w + row];
    }
  } else {
    load8(X + (int64_t)row * hw + kk, nval, v);
  }
}

template <int M>
__global__ void __launch_bounds__(256) k_tk_gram(TkTab tab, const float* __restrict__ X, float* __restrict__ part) {
  __shared__ MfmaSmemR sm;
  const int c = tk_cube(tab.bstart + tab.kind_off(TK_GRAM0 + M), tab.nc, blockIdx.x);
  if (tab.halt && tab.halt[c]) return;   // the cube has met its stopping test
  const TkGeo g = tab.geo[c];
  const int local = blockIdx.x - tab.bstart[tab.kind_off(TK_GRAM0 + M) + c];
  const int d = M == 0 ? g.h : (M == 1 ? g.w : g.b);
  const int T = (d + kMT - 1) / kMT, ntile = T * (T + 1) / 2;
  const int G = g.groups[M];
  const int tl = local % ntile, grp = local / ntile;
  int ti = 0, rem = tl;
  while (rem > ti) { rem -= ti + 1; ++ti; }
  const int tj = rem;
  const int64_t K = M == 0 ? (int64_t)g.b * g.w : (M == 1 ? (int64_t)g.b * g.h : (int64_t)g.h * g.w);
  const int64_t KG = g.kg[M];
  const int64_t k0 = (int64_t)grp * KG, k1 = (k0 + KG) < K ? (k0 + KG) : K;
  const float* Xc = X + g.off;
  const int m0 = ti * kMT, n0 = tj * kMT;
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < d && n0 + 32 * (wv & 1) < d;
  float* out = part + g.part_off[M] + ((int64_t)tl * G + grp) * (kMT * kMT);
  auto fa = [&](int m, int k, float(&v)[8]) { tk_gram_fetch<M>(Xc, g, m, k0 + k, k1, v); };
  auto fb = [&](int k, int n, float(&v)[8]) { tk_gram_fetch<M>(Xc, g, n, k0 + k, k1, v); };
  auto st = [&](int row, int col, float v) { out[(row - m0) * kMT + (col - n0)] = v; };
  constexpr bool KF = M != 1;   // the contraction index is the contiguous one
  mfma_rtile_t<KF, KF>(threadIdx.x, m0, n0, (int)(k1 - k0), fa, fb, st, sm, active);
}

// gram[packed(r, c)] = (sum over groups of the partial (r, c), 0) for the
// mode-M slice of every cube.
__global__ void __launch_bounds__(256) k_tk_reduce(TkTab tab, int M, const float* __restrict__ part,
                                                   float2* __restrict__ gram, const SliceDesc* __restrict__ hdesc) {
  const int c = tk_cube(tab.bstart + tab.kind_off(TK_RED0 + M), tab.nc, blockIdx.x);
  if (tab.halt && tab.halt[c]) return;   // the cube has met its stopping test
  const TkGeo g = tab.geo[c];
  const int local = blockIdx.x - tab.bstart[tab.kind_off(TK_RED0 + M) + c];
  const int d = M == 0 ? g.h : (M == 1 ? g.w : g.b);
  const int64_t e = (int64_t)local * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * (d + 1) / 2) return;
  const int r = packed_row(e), col = (int)(e - (int64_t)r * (r + 1) / 2);
  const int ti = r / kMT, tj = col / kMT, tl = ti * (ti + 1) / 2 + tj;
  const int G = g.groups[M];
  const float* p = part + g.part_off[M] + (int64_t)tl * G * (kMT * kMT) + (r - ti * kMT) * kMT + (col - tj * kMT);
  float s = 0.f;
  for (int q = 0; q < G; ++q) s += p[(int64_t)q * (kMT * kMT)];
  const SliceDesc sd = hdesc[M * tab.nc + c];
  gram[sd.g_off + e] = make_float2(s, 0.f);
}

// ----------------------------------------------------------- projectors ---
// P = Re(V_r V_r^H) = Vr_r Vr_r^T + Vi_r Vi_r^T, V (n x n planar, column c =
// the c-th largest eigenpair), r = rcount of the slice.
__global__ void __launch_bounds__(256) k_tk_proj(TkTab tab, int M, const SliceDesc* __restrict__ hdesc,
                                                 const float* __restrict__ V, const int* __restrict__ rcount,
                                                 float* __restrict__ P) {
  __shared__ MfmaSmemR sm;
  const int c = tk_cube(tab.bstart + tab.kind_off(TK_PROJ0 + M), tab.nc, blockIdx.x);
  if (tab.halt && tab.halt[c]) return;   // the cube has met its stopping test
  const TkGeo g = tab.geo[c];
  const int local = blockIdx.x - tab.bstart[tab.kind_off(TK_PROJ0 + M) + c];
  const int sl = M * tab.nc + c;
  const SliceDesc sd = hdesc[sl];
  const int n = sd.n1, r = rcount[sl];
  const int T = (n + kMT - 1) / kMT;
  const int m0 = (local / T) * kMT, n0 = (local % T) * kMT;
  const float* vr = V + sd.v_off;
  const float* vi = vr + (int64_t)n * n;
  float* out = P + g.p_off[M];
  const int wv = threadIdx.x >> 6;
  const bool active = m0 + 32 * (wv >> 1) < n && n0 + 32 * (wv & 1) < n;
  auto get = [&](int row, int k, float(&v)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      v[e] = (row < n && kk < 2 * r) ? (kk < r ? vr[(int64_t)row * n + kk] : vi[(int64_t)row * n + kk - r]) : 0.f;
    }
  };
  auto fa = [&](int m, int k, float(&v)[8]) { get(m, k, v); };
  auto fb = [&](int k, int nn, float(&v)[8]) { get(nn, k, v); };
  auto st = [&](int row, int col, float v) {
    if (row < n && col < n) out[(int64_t)row * n + col] = v;
  };
  mfma_rtile_t<true, true>(threadIdx.x, m0, n0, 2 * r, fa, fb, st, sm, active);
}

// --------------------------------------------------------- mode products ---
// Y = X x_M P (P symmetric d x d).  M = 0: per band, Y_j = P X_j;
// M = 1: per band, Y_j = X_j P; M = 2: Y (b x hw) = P X (b x hw).
// fin != 0 (M = 2 only): Y is the new L: T += mu (Y - L_old), L = Y.
template <int M>
__global__ void __launch_bounds__(256) k_tk_prod(TkTab tab, const float* __restrict__ X, const float* __restrict__ P,
                                                 float* __restrict__ Y, float* __restrict__ Lc, float* __restrict__ Tz,
                                                 const double* __restrict__ mu_dev, int fin) {
  __shared__ MfmaSmemR sm;
  const int c = tk_cube(tab.bstart + tab.kind_off(TK_PROD0 + M), tab.nc, blockIdx.x);
  if (tab.halt && tab.halt[c]) return;   // the cube has met its stopping test
  const TkGeo g = tab.geo[c];
  const int local = blockIdx.x - tab.bstart[tab.kind_off(TK_PROD0 + M) + c];
  const int h = g.h, w = g.w, b = g.b;
  const int64_t hw = (int64_t)h * w;
  const float* Pm = P + g.p_off[M];
  const int wv = threadIdx.x >> 6;
  if (M == 0 || M == 1) {
    const int TH = (h + kMT - 1) / kMT, TW = (w + kMT - 1) / kMT;
    const int j = local / (TH * TW), rem = local - j * TH * TW;
    const int m0 = (rem / TW) * kMT, n0 = (rem % TW) * kMT;
    const float* Xj = X + g.off + (int64_t)j * hw;
    float* Yj = Y + g.off + (int64_t)j * hw;
    const bool active = m0 + 32 * (wv >> 1) < h && n0 + 32 * (wv & 1) < w;
    const int K = M == 0 ? h : w;
    // A (h x K): M = 0: P (row-major h x h); M = 1: X_j (row-major h x w)
    auto fa = [&](int m, int k, float(&v)[8]) {
      const int nv = m < h ? (K - k < 8 ? K - k : 8) : 0;
      if (nv <= 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
        return;
      }
      load8((M == 0 ? Pm + (int64_t)m * h : Xj + (int64_t)m * w) + k, nv, v);
    };
    // B (K x w), four-wide along n: M = 0: X_j; M = 1: P (w x w)
    auto fb = [&](int k, int n, float(&v)[4]) {
      const int nv = k < K ? (w - n < 4 ? w - n : 4) : 0;
      if (nv <= 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = 0.f;
        return;
      }
      load4((M == 0 ? Xj : Pm) + (int64_t)k * w + n, nv, v);
    };
    auto st = [&](int row, int col, float v) {
      if (row < h && col < w) Yj[(int64_t)row * w + col] = v;
    };
    mfma_rtile_t<true, false, true>(threadIdx.x, m0, n0, K, fa, fb, st, sm, active);
  } else {
    const int TN = (int)((hw + kMT - 1) / kMT);
    const int m0 = (local / TN) * kMT, n0 = (local % TN) * kMT;   // hw <= 512 * 512 fits int
    const float* Xc = X + g.off;
    const bool active = m0 + 32 * (wv >> 1) < b && n0 + 32 * (wv & 1) < hw;
    const float mu = fin ? (float)(*mu_dev) : 0.f;
    auto fa = [&](int m, int k, float(&v)[8]) {
      const int nv = m < b ? (b - k < 8 ? b - k : 8) : 0;
      if (nv <= 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
        return;
      }
      load8(Pm + (int64_t)m * b + k, nv, v);
    };
    auto fb = [&](int k, int n, float(&v)[4]) {
      const int nv = k < b ? (int)(hw - n < 4 ? hw - n : 4) : 0;
      if (nv <= 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = 0.f;
        return;
      }
      load4(Xc + (int64_t)k * hw + n, nv, v);
    };
    auto st = [&](int row, int col, float v) {
      if (row < b && col < hw) {
        const int64_t q = g.off + (int64_t)row * hw + col;
        if (fin) {
          const float old = Lc[q];
          Tz[q] += mu * (v - old);
          Lc[q] = v;
        } else {
          Y[q] = v;
        }
      }
    };
    mfma_rtile_t<true, false, true>(threadIdx.x, m0, n0, b, fa, fb, st, sm, active);
  }
}

// ------------------------------------------------------------- launchers ---
void launch_tk_gram(const TkTab& tab, int M, const float* X, float* part, hipStream_t s) {
  const int nb = tab.nblocks[TK_GRAM0 + M];
  if (nb == 0) return;
  if (M == 0) hipLaunchKernelGGL(k_tk_gram<0>, dim3(nb), dim3(256), 0, s, tab, X, part);
  else if (M == 1) hipLaunchKernelGGL(k_tk_gram<1>, dim3(nb), dim3(256), 0, s, tab, X, part);
  else hipLaunchKernelGGL(k_tk_gram<2>, dim3(nb), dim3(256), 0, s, tab, X, part);
}

void launch_tk_reduce(const TkTab& tab, int M, const float* part, float2* gram, const SliceDesc* hdesc,
                      hipStream_t s) {
  const int nb = tab.nblocks[TK_RED0 + M];
  if (nb == 0) return;
  hipLaunchKernelGGL(k_tk_reduce, dim3(nb), dim3(256), 0, s, tab, M, part, gram, hdesc);
}

void launch_tk_proj(const TkTab& tab, int M, const SliceDesc* hdesc, const float* V, const int* rcount, float* P,
                    hipStream_t s) {
  const int nb = tab.nblocks[TK_PROJ0 + M];
  if (nb == 0) return;
  hipLaunchKernelGGL(k_tk_proj, dim3(nb), dim3(256), 0, s, tab, M, hdesc, V, rcount, P);
}

void launch_tk_prod(const TkTab& tab, int M, const float* X, const float* P, float* Y, float* L, float* T,
                    const double* mu, bool fin, hipStream_t s) {
  const int nb = tab.nblocks[TK_PROD0 + M];
  if (nb == 0) return;
  if (M == 0) hipLaunchKernelGGL(k_tk_prod<0>, dim3(nb), dim3(256), 0, s, tab, X, P, Y, L, T, mu, 0);
  else if (M == 1) hipLaunchKernelGGL(k_tk_prod<1>, dim3(nb), dim3(256), 0, s, tab, X, P, Y, L, T, mu, 0);
  else hipLaunchKernelGGL(k_tk_prod<2>, dim3(nb), dim3(256), 0, s, tab, X, P, Y, L, T, mu, fin ? 1 : 0);
}

}  // namespace lrstv
