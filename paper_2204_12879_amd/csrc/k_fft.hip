// Transforms of the ADMM sweep.
//
// Z-update (Sec. III-C): the system mu (I + sum_n w_n^2 D_n^T D_n) Z = T_z is
// diagonalised by DFTs along the two spatial axes (the paper's fftn route);
// what remains for every spatial frequency (k_h, k_w) is a periodic
// tridiagonal system along the bands,
//     [a I + beta C] z = t,   C = circulant(2, -1, ..., -1),
//     a = mu (1 + w_1^2 4 sin^2(pi k_h / h) + w_2^2 4 sin^2(pi k_w / w)),
//     beta = mu w_3^2,
// whose solution equals the band DFT route exactly (up to rounding).  It is
// solved in O(b) with the factorisation a + 2 beta - beta (S + S^-1) =
// (beta / r)(1 - r S)(1 - r S^-1), 0 < r < 1, i.e. one causal and one
// anti-causal periodic first-order recursion.  This avoids an FFT of prime
// length along the bands (b = 191 for the 256x256x191 cube).
//
// t-SVT (Sec. III-C E-update): real DFT along the bands of each gradient
// tensor into the floor(b/2)+1 non-redundant frontal slices, and the inverse
// with conjugate-symmetric completion, fused with the Gamma4 ascent.
//
// FFTs along w and h run in LDS as batched Stockham autosort transforms with
// radices 4, 2, 3, 5, 7 and a direct-DFT stage for any other prime factor.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace lrstv {

#define MAX_STAGES 24
constexpr int kFftHThreads = 512;  // a multiple of every column count cw <= 16
// The inverse w transform has one block per residual slot (LRSTV_PARTS per
// cube), so it takes large blocks to keep enough waves in flight.
constexpr int kIrfftThreads = 512;

struct Plan {
  int ns;
  int r[MAX_STAGES];
};

LRSTV_DEV void make_plan(int N, Plan& p) {
  p.ns = 0;
  int n = N;
  const int small[5] = {4, 2, 3, 5, 7};
  for (int t = 0; t < 5; ++t)
    while (n % small[t] == 0 && p.ns < MAX_STAGES) {
      p.r[p.ns++] = small[t];
      n /= small[t];
    }
  for (int q = 11; n > 1 && p.ns < MAX_STAGES; q += 2)
    while (n % q == 0) {
      p.r[p.ns++] = q;
      n /= q;
    }
}

// tw[m] = exp(-2 pi i m / N)
LRSTV_DEV void fill_twiddles(float2* tw, int N) {
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
  }
}

LRSTV_DEV float2 twid(const float2* tw, int m, int sign) {
  const float2 t = tw[m];
  return sign < 0 ? t : make_float2(t.x, -t.y);
}

template <int R>
LRSTV_DEV void small_dft(float2* v, const float2* tw, int N, int sign) {
  if (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    const float2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = csub(a1, a3);
    // -i * d13 for the forward transform (sign < 0), +i * d13 for the inverse
    const float2 rot = sign < 0 ? make_float2(d13.y, -d13.x) : make_float2(-d13.y, d13.x);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, rot);
    v[3] = csub(d02, rot);
  } else {
    // the R-th roots read once; (q s) mod R is a constant of the unrolled loops
    float2 wr[R];
    const int step = N / R;
#pragma unroll
    for (int j = 1; j < R; ++j) wr[j] = twid(tw, j * step, sign);
    float2 o[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
      float2 acc = v[0];
#pragma unroll
      for (int q = 1; q < R; ++q) acc = (q * s) % R == 0 ? cadd(acc, v[q]) : cadd(acc, cmul(v[q], wr[(q * s) % R]));
      o[s] = acc;
    }
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = o[s];
  }
}

template <int R>
LRSTV_DEV void stage_small(const float2* src, float2* dst, int N, int ld, int nb, int Ns, const float2* tw, int sign) {
  const int NR = N / R;
  const int tot = nb * NR;
  const int tstep = N / (Ns * R);
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int f = t / NR, j = t - f * NR, k = j % Ns;
    const float2* s = src + f * ld;
    float2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v[q] = s[j + q * NR];
      if (q > 0 && k > 0) v[q] = cmul(v[q], twid(tw, q * k * tstep, sign));
    }
    small_dft<R>(v, tw, N, sign);
    const int idx = (j / Ns) * Ns * R + k;
    float2* d = dst + f * ld + idx;
#pragma unroll
    for (int q = 0; q < R; ++q) d[q * Ns] = v[q];
  }
}

// Direct DFT stage for a prime factor R > 7.  Outputs so and R - so of one
// butterfly share the input reads, the input twiddles and the root read
// (w^(q (R - so)) = conj(w^(q so))): a thread forms both.
LRSTV_DEV void stage_generic(const float2* src, float2* dst, int N, int ld, int nb, int Ns, int R, const float2* tw,
                             int sign) {
  const int NR = N / R, H = (R + 1) / 2, per = NR * H;
  const int tstep = N / (Ns * R), ostep = N / R;
  for (int t = threadIdx.x; t < nb * per; t += blockDim.x) {
    const int f = t / per, rem = t - f * per;
    const int so = rem / NR, j = rem - so * NR;   // j = jd Ns + k
    const int k = j % Ns, jd = j / Ns;
    const float2* s = src + f * ld;
    float2 p = make_float2(0.f, 0.f), m = make_float2(0.f, 0.f);   // X_so, X_(R-so)
    int oi = 0;  // (q * so) mod R
    for (int q = 0; q < R; ++q) {
      float2 a = s[j + q * NR];
      if (q > 0 && k > 0) a = cmul(a, twid(tw, q * k * tstep, sign));
      const float2 w = twid(tw, oi * ostep, sign);
      const float rr = a.x * w.x, ii = a.y * w.y, ri = a.x * w.y, ir = a.y * w.x;
      p.x += rr - ii;
      p.y += ri + ir;
      m.x += rr + ii;
      m.y += ir - ri;
      oi += so;
      if (oi >= R) oi -= R;
    }
    float2* d = dst + f * ld + jd * Ns * R + k;
    d[so * Ns] = p;
    if (so > 0) d[(R - so) * Ns] = m;
  }
}

// Batched FFT of nb rows of length N held in bufA at row stride ld; returns
// the buffer holding the result.  Unnormalised; sign -1 forward, +1 inverse.
LRSTV_DEV float2* fft_lds(float2* bufA, float2* bufB, int N, int ld, int nb, const float2* tw, int sign,
                          const Plan& p) {
  float2* src = bufA;
  float2* dst = bufB;
  int Ns = 1;
  for (int st = 0; st < p.ns; ++st) {
    const int R = p.r[st];
    switch (R) {
      case 2: stage_small<2>(src, dst, N, ld, nb, Ns, tw, sign); break;
      case 3: stage_small<3>(src, dst, N, ld, nb, Ns, tw, sign); break;
      case 4: stage_small<4>(src, dst, N, ld, nb, Ns, tw, sign); break;
      case 5: stage_small<5>(src, dst, N, ld, nb, Ns, tw, sign); break;
      case 7: stage_small<7>(src, dst, N, ld, nb, Ns, tw, sign); break;
      default: stage_generic(src, dst, N, ld, nb, Ns, R, tw, sign); break;
    }
    __syncthreads();
    float2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// ---------------------------------------------------------------------------
// Real FFT along w, two rows packed in one complex transform.
// T: rows r = j*h + i of length w; spec rows of length wc = w/2 + 1.
LRSTV_DEV void rfft_w_body(int bid, int nblk, float2* sm, const float* __restrict__ T, float2* __restrict__ spec, int nrows,
                                                int w, int nb) {
  float2* tw = sm;
  float2* bA = sm + w;
  float2* bB = bA + nb * w;
  const int wc = w / 2 + 1;
  Plan p;
  make_plan(w, p);
  fill_twiddles(tw, w);
  const int rows_per_block = 2 * nb;
  for (int r0 = bid * rows_per_block; r0 < nrows; r0 += nblk * rows_per_block) {
    for (int t = threadIdx.x; t < nb * w; t += blockDim.x) {
      const int f = t / w, x = t - f * w;
      const int ra = r0 + 2 * f, rb = ra + 1;
      const float va = ra < nrows ? T[(int64_t)ra * w + x] : 0.f;
      const float vb = rb < nrows ? T[(int64_t)rb * w + x] : 0.f;
      bA[t] = make_float2(va, vb);
    }
    __syncthreads();
    const float2* out = fft_lds(bA, bB, w, w, nb, tw, -1, p);
    for (int t = threadIdx.x; t < nb * wc; t += blockDim.x) {
      const int f = t / wc, k = t - f * wc;
      const float2 zk = out[f * w + k];
      const float2 zc = cconj(out[f * w + ((w - k) % w)]);
      const float2 X = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      const float2 D = csub(zk, zc);                 // Y = D / (2i)
      const float2 Y = make_float2(0.5f * D.y, -0.5f * D.x);
      const int ra = r0 + 2 * f, rb = ra + 1;
      if (ra < nrows) spec[(int64_t)ra * wc + k] = X;
      if (rb < nrows) spec[(int64_t)rb * wc + k] = Y;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_rfft_w(const float* __restrict__ T, float2* __restrict__ spec, int nrows,
                                                int w, int nb) {
  extern __shared__ float2 sm[];
  rfft_w_body(blockIdx.x, gridDim.x, sm, T, spec, nrows, w, nb);
}

// Inverse of k_rfft_w (scaled by `scale`), writing real rows into Z.  If
// `part` is set, also accumulates sum (Z_new - Z_old)^2 per block.
LRSTV_DEV void irfft_w_body(int bid, int nblk, float2* sm, const float2* __restrict__ spec, float* __restrict__ Z, int nrows,
                                                 int w, int nb, float scale, double* __restrict__ part) {
  __shared__ double red[kIrfftThreads / 64];
  float2* tw = sm;
  float2* bA = sm + w;
  float2* bB = bA + nb * w;
  const int wc = w / 2 + 1;
  Plan p;
  make_plan(w, p);
  fill_twiddles(tw, w);
  double acc = 0.0;
  const int rows_per_block = 2 * nb;
  for (int r0 = bid * rows_per_block; r0 < nrows; r0 += nblk * rows_per_block) {
    for (int t = threadIdx.x; t < nb * w; t += blockDim.x) {
      const int f = t / w, k = t - f * w;
      const int ra = r0 + 2 * f, rb = ra + 1;
      const bool lo = k < wc;
      const int kk = lo ? k : w - k;
      float2 X = ra < nrows ? spec[(int64_t)ra * wc + kk] : make_float2(0.f, 0.f);
      float2 Y = rb < nrows ? spec[(int64_t)rb * wc + kk] : make_float2(0.f, 0.f);
      if (!lo) {
        X = cconj(X);
        Y = cconj(Y);
      }
      bA[t] = make_float2(X.x - Y.y, X.y + Y.x);  // X + i Y
    }
    __syncthreads();
    const float2* out = fft_lds(bA, bB, w, w, nb, tw, +1, p);
    for (int t = threadIdx.x; t < nb * w; t += blockDim.x) {
      const int f = t / w, x = t - f * w;
      const int ra = r0 + 2 * f, rb = ra + 1;
      const float2 v = out[t];
      if (ra < nrows) {
        const int64_t q = (int64_t)ra * w + x;
        const float zn = v.x * scale;
        if (part) {
          const double d = (double)zn - (double)Z[q];
          acc += d * d;
        }
        Z[q] = zn;
      }
      if (rb < nrows) {
        const int64_t q = (int64_t)rb * w + x;
        const float zn = v.y * scale;
        if (part) {
          const double d = (double)zn - (double)Z[q];
          acc += d * d;
        }
        Z[q] = zn;
      }
    }
    __syncthreads();
  }
  if (part) {
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[R_DUAL_Z * LRSTV_PARTS + bid] = acc;
  }
}

__global__ void __launch_bounds__(kIrfftThreads) k_irfft_w(const float2* __restrict__ spec, float* __restrict__ Z, int nrows,
                                                 int w, int nb, float scale, double* __restrict__ part) {
  extern __shared__ float2 sm[];
  irfft_w_body(blockIdx.x, gridDim.x, sm, spec, Z, nrows, w, nb, scale, part);
}

// Complex FFT along h of spec [b][h][wc].  The b * wc columns are taken as
// one flat list, cw consecutive ones per block (a block reads whole 128-byte
// row segments and no column is wasted at a band edge).  In LDS each column
// is a row of stride ld = h + ((2 - h) mod 32): ld = 2 (mod 32) makes the
// transposing loads and stores free of bank conflicts.
LRSTV_DEV int fft_h_ld(int h) { return h + (((2 - h) % 32) + 32) % 32; }

LRSTV_DEV void fft_h_body(int bid, int nblk, float2* sm, float2* __restrict__ spec, int h, int wc, int b, int cw, int sign) {
  const int ld = fft_h_ld(h);
  float2* tw = sm;
  float2* bA = sm + h;
  float2* bB = bA + cw * ld;
  Plan p;
  make_plan(h, p);
  fill_twiddles(tw, h);
  const int64_t ncol = (int64_t)b * wc, plane = (int64_t)h * wc;
  const int64_t nchunk = (ncol + cw - 1) / cw;
  // blockDim is a multiple of cw, so a thread keeps its column f
  const int f = threadIdx.x % cw, i0 = threadIdx.x / cw, di = blockDim.x / cw;
  for (int64_t blk = xcd_block(bid, nblk); blk < nchunk; blk += nblk) {
    const int64_t g = blk * cw + f;
    const bool ok = g < ncol;
    const int64_t j = ok ? g / wc : 0;
    float2* base = spec + j * plane + (ok ? g - j * wc : 0);
    for (int i = i0; i < h; i += di) bA[f * ld + i] = ok ? base[(int64_t)i * wc] : make_float2(0.f, 0.f);
    __syncthreads();
    const float2* out = fft_lds(bA, bB, h, ld, cw, tw, sign, p);
    if (ok)
      for (int i = i0; i < h; i += di) base[(int64_t)i * wc] = out[f * ld + i];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kFftHThreads) k_fft_h(float2* __restrict__ spec, int h, int wc, int b, int cw, int sign) {
  extern __shared__ float2 sm[];
  fft_h_body(blockIdx.x, gridDim.x, sm, spec, h, wc, b, cw, sign);
}

// ------------------------------------------------- register FFT along h ---
// For h = P Q with P, Q in {8, 16} (h = 64, 128, 256) the column transforms
// run in registers: with n = Q p + q and k = k1 + P k2,
//   X[k1 + P k2] = sum_q w_Q^(q k2) w_h^(q k1) sum_p x[Q p + q] w_P^(p k1),
// thread (column, q) forms the inner P-point DFT of its column's elements
// Q p + q, multiplies by w_h^(q k1) and writes them to LDS; after one barrier
// thread (column, k1) reads the Q values y[q][k1] and forms the outer
// Q-point DFT, writing X[k1 + P k2].  Two passes over LDS per transform
// instead of one per Stockham stage.  The in-register DFTs split R = A B the
// same way (down to radix 2).  Unnormalised; S = -1 forward, +1 inverse.
__constant__ constexpr float kCos16[16] = {1.f, 0.9238795325f, 0.7071067812f, 0.3826834324f, 0.f, -0.3826834324f,
                                           -0.7071067812f, -0.9238795325f, -1.f, -0.9238795325f, -0.7071067812f,
                                           -0.3826834324f, 0.f, 0.3826834324f, 0.7071067812f, 0.9238795325f};
__constant__ constexpr float kSin16[16] = {0.f, 0.3826834324f, 0.7071067812f, 0.9238795325f, 1.f, 0.9238795325f,
                                           0.7071067812f, 0.3826834324f, 0.f, -0.3826834324f, -0.7071067812f,
                                           -0.9238795325f, -1.f, -0.9238795325f, -0.7071067812f, -0.3826834324f};

template <int R, int S>
LRSTV_DEV void dft_reg(float2 (&v)[R]) {
  if constexpr (R == 2) {
    const float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else {
    constexpr int A = (R == 4) ? 2 : 4, B = R / A;   // n = B n1 + n2, k = k1 + A k2
    float2 t[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      float2 u[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) u[n1] = v[B * n1 + n2];
      dft_reg<A, S>(u);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int m = (n2 * k1) % R;   // w_R^(n2 k1)
        t[n2][k1] = m == 0 ? u[k1] : cmul(u[k1], make_float2(kCos16[m * (16 / R)], S * kSin16[m * (16 / R)]));
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      float2 u[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) u[n2] = t[n2][k1];
      dft_reg<B, S>(u);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k2];
    }
  }
}

constexpr int kFftRegCols = 32;   // columns per block (two 128-byte row segments)
template <int P, int Q>
constexpr int fft_reg_threads() { return kFftRegCols * (P > Q ? P : Q); }

template <int P, int Q, int S>
LRSTV_DEV void fft_h_reg_body(int bid, int nblk, float2* __restrict__ spec, int wc, int b) {
  constexpr int N = P * Q, C = kFftRegCols;
  __shared__ float2 Y[P][Q][C];
  __shared__ float2 tw[N];   // w_N^m
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double sv, cv;
    sincospi(2.0 * (double)m / (double)N, &sv, &cv);
    tw[m] = make_float2((float)cv, (float)(S * sv));
  }
  const int c = threadIdx.x % C, rr = threadIdx.x / C;
  const int64_t ncol = (int64_t)b * wc, plane = (int64_t)N * wc;
  const int64_t nchunk = (ncol + C - 1) / C;
  for (int64_t blk = xcd_block(bid, nblk); blk < nchunk; blk += nblk) {
    const int64_t g = blk * C + c;
    const bool ok = g < ncol;
    const int64_t j = ok ? g / wc : 0;
    float2* base = spec + j * plane + (ok ? g - j * wc : 0);
    __syncthreads();   // the twiddle table (first pass) and the previous pass's reads of Y
    if (rr < Q) {
      float2 v[P];
#pragma unroll
      for (int p = 0; p < P; ++p) v[p] = ok ? base[(int64_t)(Q * p + rr) * wc] : make_float2(0.f, 0.f);
      dft_reg<P, S>(v);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) Y[k1][rr][c] = k1 == 0 ? v[0] : cmul(v[k1], tw[rr * k1]);
    }
    __syncthreads();
    if (rr < P) {
      float2 u[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) u[q] = Y[rr][q][c];
      dft_reg<Q, S>(u);
      if (ok) {
#pragma unroll
        for (int k2 = 0; k2 < Q; ++k2) base[(int64_t)(rr + P * k2) * wc] = u[k2];
      }
    }
  }
}

template <int P, int Q, int S>
__global__ void __launch_bounds__(kFftRegCols * (P > Q ? P : Q)) k_fft_h_reg(float2* __restrict__ spec, int wc, int b) {
  fft_h_reg_body<P, Q, S>(blockIdx.x, gridDim.x, spec, wc, b);
}


// ---------------------------------------------- register real FFTs along w ---
// Two real rows a, b of length w = P Q (64, 128, 256) as one complex
// transform z = a + i b, computed as the h transform above (16 threads per
// row pair).  Forward: A[k] = (Z[k] + conj Z[w-k]) / 2,
// B[k] = (Z[k] - conj Z[w-k]) / (2 i) for k <= w/2 (Z goes through LDS for the
// mirrored index).  Inverse: Z[k] = A[k] + i B[k] with A[w-k] = conj A[k];
// a = Re z, b = Im z, times `scale`, into Z, with the FP64 partial of
// (Z_new - Z_old)^2 when `part` is set.
constexpr int kPairThreads = 16;
template <int PPB, int P, int Q, int S>
struct RowFft {
  static constexpr int N = P * Q;
  float2 Y[PPB][N];   // the pair's y[q][k1] at k1 * Q + q, then Z[k] at k
  float2 tw[N];
};

template <int P, int Q, int S, int PPB>
LRSTV_DEV void row_fft_inner(RowFft<PPB, P, Q, S>& sm, int f, int r, const float2 (&in)[P], float2 (&out)[Q]) {
  // first pass (threads r < Q): in = z[Q p + r]; second (threads r < P): out = Z[r + P k2]
  constexpr int N = P * Q;
  if (r < Q) {
    float2 v[P];
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = in[p];
    dft_reg<P, S>(v);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) sm.Y[f][k1 * Q + r] = k1 == 0 ? v[0] : cmul(v[k1], sm.tw[r * k1]);
  }
  __syncthreads();
  if (r < P) {
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = sm.Y[f][r * Q + q];
    dft_reg<Q, S>(out);
  }
  (void)N;
}

template <int P, int Q, int PPB>
LRSTV_DEV void rfft_w_reg_body(int bid, int nblk, const float* __restrict__ T, float2* __restrict__ spec, int nrows) {
  constexpr int N = P * Q, wc = N / 2 + 1;
  __shared__ RowFft<PPB, P, Q, -1> sm;
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double sv, cv;
    sincospi(2.0 * (double)m / (double)N, &sv, &cv);
    sm.tw[m] = make_float2((float)cv, (float)(-sv));
  }
  const int f = threadIdx.x / kPairThreads, r = threadIdx.x % kPairThreads;
  const int npairs = (nrows + 1) / 2;
  for (int pb = bid * PPB; pb < npairs; pb += nblk * PPB) {
    const int pair = pb + f, ra = 2 * pair, rb = ra + 1;
    const bool oka = pair < npairs, okb = rb < nrows;
    float2 in[P], out[Q];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int n = Q * p + r;
      in[p] = make_float2(oka && r < Q ? T[(int64_t)ra * N + n] : 0.f, okb && r < Q ? T[(int64_t)rb * N + n] : 0.f);
    }
    __syncthreads();   // twiddles ready, previous pair block's reads of Y done
    row_fft_inner<P, Q, -1, PPB>(sm, f, r, in, out);
    __syncthreads();
    if (r < P) {
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) sm.Y[f][r + P * k2] = out[k2];
    }
    __syncthreads();
    for (int k = r; k < wc; k += kPairThreads) {
      const float2 zk = sm.Y[f][k];
      const float2 zc = cconj(sm.Y[f][(N - k) % N]);
      const float2 A = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      const float2 D = csub(zk, zc);
      const float2 B = make_float2(0.5f * D.y, -0.5f * D.x);
      if (oka) spec[(int64_t)ra * wc + k] = A;
      if (okb) spec[(int64_t)rb * wc + k] = B;
    }
  }
}

template <int P, int Q, int PPB>
LRSTV_DEV void irfft_w_reg_body(int bid, int nblk, const float2* __restrict__ spec, float* __restrict__ Z, int nrows,
                                float scale, double* __restrict__ part) {
  constexpr int N = P * Q, wc = N / 2 + 1;
  __shared__ RowFft<PPB, P, Q, 1> sm;
  __shared__ double red[PPB * kPairThreads / 64];
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double sv, cv;
    sincospi(2.0 * (double)m / (double)N, &sv, &cv);
    sm.tw[m] = make_float2((float)cv, (float)sv);
  }
  const int f = threadIdx.x / kPairThreads, r = threadIdx.x % kPairThreads;
  const int npairs = (nrows + 1) / 2;
  double acc = 0.0;
  for (int pb = bid * PPB; pb < npairs; pb += nblk * PPB) {
    const int pair = pb + f, ra = 2 * pair, rb = ra + 1;
    const bool oka = pair < npairs, okb = rb < nrows;
    float2 in[P], out[Q];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int n = Q * p + r;
      const bool lo = n <= N / 2;
      const int kk = lo ? n : N - n;
      float2 X = (oka && r < Q) ? spec[(int64_t)ra * wc + kk] : make_float2(0.f, 0.f);
      float2 Yb = (okb && r < Q) ? spec[(int64_t)rb * wc + kk] : make_float2(0.f, 0.f);
      if (!lo) {
        X = cconj(X);
        Yb = cconj(Yb);
      }
      in[p] = make_float2(X.x - Yb.y, X.y + Yb.x);   // X + i Y
    }
    __syncthreads();
    row_fft_inner<P, Q, 1, PPB>(sm, f, r, in, out);
    if (r < P) {
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) {
        const int x = r + P * k2;
        if (oka) {
          const int64_t q = (int64_t)ra * N + x;
          const float zn = out[k2].x * scale;
          if (part) {
            const double d = (double)zn - (double)Z[q];
            acc += d * d;
          }
          Z[q] = zn;
        }
        if (okb) {
          const int64_t q = (int64_t)rb * N + x;
          const float zn = out[k2].y * scale;
          if (part) {
            const double d = (double)zn - (double)Z[q];
            acc += d * d;
          }
          Z[q] = zn;
        }
      }
    }
  }
  if (part) {
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[R_DUAL_Z * LRSTV_PARTS + bid] = acc;
  }
}

constexpr int kRfftPairs = 16, kIrfftPairs = 32;   // row pairs per block

// Periodic tridiagonal solve along the bands for every (k_h, k_w).
//
// A block takes kTriCols columns with consecutive k_w (each band row of the
// block is then one coalesced segment) and splits every column's b bands
// into kTriChunks chunks of L = ceil(b / kTriChunks), one chunk per thread,
// held in registers: the half spectrum is read and written once.  Each
// periodic first-order recursion x_j = s_j + r x_{j -/+ 1} runs as a chunked
// scan: a local pass with zero carry gives u_j and the chunk's end value;
// the end values are exchanged through LDS; the carry into chunk q follows
// in FP64 from the periodic closure
//   x_{-1} (1 - r^b) = sum_q E_q r^(b - j1_q)         (causal pass),
//   x_b    (1 - r^b) = sum_q F_q r^(j0_q)             (anti-causal pass),
// propagated chunk by chunk, and x_j = u_j + r^d C with d the distance to
// the chunk's carry end.
constexpr int kTriCols = 32, kTriChunks = 16;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// r^k for k >= 0 by binary powering (a few FP64 roundings)
LRSTV_DEV double pow_int(double r, int k) {
  double p = 1.0;
  while (k > 0) {
    if (k & 1) p *= r;
    r *= r;
    k >>= 1;
  }
  return p;
}

LRSTV_DEV double tri_chunk_pow(int q, int L, int b, double rL, double rlast) {
  const int len = min(b - q * L, L);
  return len <= 0 ? 1.0 : (len == L ? rL : rlast);
}

template <int MAXL>
LRSTV_DEV void tri_b_body(int bid, int nblk, float2* __restrict__ spec, int h, int w, int b, double w1, double w2,
                          double w3, const double* __restrict__ mu_dev, double mu_host) {
  __shared__ float2 sE[kTriChunks][kTriCols], sF[kTriChunks][kTriCols];
  const int wc = w / 2 + 1;
  const int64_t plane = (int64_t)h * wc;
  const double mu = mu_dev ? *mu_dev : mu_host;
  const double beta = mu * w3 * w3;
  const int cl = threadIdx.x % kTriCols, q = threadIdx.x / kTriCols;
  const int L = (b + kTriChunks - 1) / kTriChunks;
  const int j0 = min(q * L, b), len = min(j0 + L, b) - j0;
  const int64_t ngroups = (plane + kTriCols - 1) / kTriCols;
  // The cube's half spectrum (< 2^31 bytes for sides up to 512) is addressed
  // as a raw buffer: an element outside the chunk gets an offset beyond the
  // buffer, whose load returns 0 and whose store is dropped, so the chunk
  // loops need no per-element branches.
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(spec, 0, (int)(plane * b * (int64_t)sizeof(float2)), 0x00020000);
  const int kOut = 0x7ffffff0, pl8 = (int)(plane * (int64_t)sizeof(float2));
  for (int64_t grp = bid; grp < ngroups; grp += nblk) {
    const int64_t col = grp * kTriCols + cl;
    const bool ok = col < plane;
    const int i = ok ? (int)(col / wc) : 0, kw = ok ? (int)(col - (int64_t)i * wc) : 0;
    const double sh = sinpi((double)i / h), sw = sinpi((double)kw / w);
    const double a = mu * (1.0 + 4.0 * (w1 * w1 * sh * sh + w2 * w2 * sw * sw));
    const int n = ok ? len : 0;
    const bool rec = beta > 0.0 && b > 1;  // uniform over the launch
    double r = 0.0, rL = 0.0, rlast = 0.0, inv = 1.0;
    if (rec) {
      const double cc = (a + 2.0 * beta) / (2.0 * beta);
      r = 1.0 / (cc + sqrt(cc * cc - 1.0));
      rL = pow_int(r, L);
      rlast = pow_int(r, b - (b - 1) / L * L);
      inv = 1.0 / (1.0 - pow_int(r, b));
    }
    int base = (int)((col + (int64_t)j0 * plane) * (int64_t)sizeof(float2));
    // the loads wait for the coefficients, so that the temporaries of their
    // evaluation are not live beside the chunk
    asm volatile("" : "+v"(base) : "v"(r), "v"(rL), "v"(rlast), "v"(inv), "v"(a));
    // element e of the chunk is at byte base + e * pl8; the offset is stepped
    // in a register that is opaque to the optimiser, so that no table of
    // MAXL addresses stays live from the loads to the stores
    float2 v[MAXL];
    int off = base;
#pragma unroll
    for (int e = 0; e < MAXL; ++e) {
      const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(rs, e < n ? off : kOut, 0, 0);
      v[e] = make_float2(__uint_as_float(x.x), __uint_as_float(x.y));
      off = opaque_i(off + pl8);
    }
    auto store = [&](int e, int o, float2 z) {
      const u32x2 x = {__float_as_uint(z.x), __float_as_uint(z.y)};
      __builtin_amdgcn_raw_buffer_store_b64(x, rs, e < n ? o : kOut, 0, 0);
    };
    if (!rec) {  // no recursion along the bands
      const float ia = (float)(1.0 / a);
      off = base;
#pragma unroll
      for (int e = 0; e < MAXL; ++e) {
        store(e, off, cscale(v[e], ia));
        off = opaque_i(off + pl8);
      }
      continue;
    }
    const float rf = (float)r;
    // causal: y_j = t_j + r y_{j-1}; u holds the chunk's end value
    float2 u = make_float2(0.f, 0.f);
#pragma unroll
    for (int e = 0; e < MAXL; ++e) {
      const float2 y = make_float2(fmaf(rf, u.x, v[e].x), fmaf(rf, u.y, v[e].y));
      u = e < n ? y : u;
      v[e] = y;
    }
    sE[q][cl] = u;
    __syncthreads();
    // one pass over the end values: S = sum_p E_p r^(b - j1_p) (closure),
    // T = sum_{p<q} E_p r^(j0_q - j1_p), R = r^(j0_q); C_q = T + R y_{-1}
    double sx = 0.0, sy = 0.0, tx = 0.0, ty = 0.0, R = 1.0;
#pragma unroll
    for (int p = 0; p < kTriChunks; ++p) {
      const double P = tri_chunk_pow(p, L, b, rL, rlast);
      const float2 E = sE[p][cl];
      sx = sx * P + E.x;
      sy = sy * P + E.y;
      if (p < q) {
        tx = tx * P + E.x;
        ty = ty * P + E.y;
        R *= P;
      }
    }
    const double cx = tx + R * (sx * inv), cy = ty + R * (sy * inv);
    double pe = r;
#pragma unroll
    for (int e = 0; e < MAXL; ++e) {
      v[e] = make_float2(v[e].x + (float)(pe * cx), v[e].y + (float)(pe * cy));
      pe *= r;
    }
    // anti-causal: z_j = y_j + r z_{j+1}; u holds the chunk's start value
    u = make_float2(0.f, 0.f);
#pragma unroll
    for (int e = MAXL - 1; e >= 0; --e) {
      const float2 z = make_float2(fmaf(rf, u.x, v[e].x), fmaf(rf, u.y, v[e].y));
      u = e < n ? z : make_float2(0.f, 0.f);
      v[e] = u;
    }
    sF[q][cl] = u;
    __syncthreads();
    // S = sum_p F_p r^(j0_p), T = sum_{p>q} F_p r^(j0_p - j1_q),
    // R = r^(b - j1_q); D_q = z_{j1_q} = T + R z_b, z_b = z_0
    sx = sy = tx = ty = 0.0;
    R = 1.0;
#pragma unroll
    for (int p = kTriChunks - 1; p >= 0; --p) {
      const double P = tri_chunk_pow(p, L, b, rL, rlast);
      const float2 F = sF[p][cl];
      sx = sx * P + F.x;
      sy = sy * P + F.y;
      if (p > q) {
        tx = tx * P + F.x;
        ty = ty * P + F.y;
        R *= P;
      }
    }
    const double dx = tx + R * (sx * inv), dy = ty + R * (sy * inv);
    const float sc = (float)(r / beta);
    pe = r;  // r^(j1 - j) at element j; held at r above the chunk's end
    off = opaque_i(base + (MAXL - 1) * pl8);
#pragma unroll
    for (int e = MAXL - 1; e >= 0; --e) {
      const float2 z = make_float2(v[e].x + (float)(pe * dx), v[e].y + (float)(pe * dy));
      store(e, off, cscale(z, sc));
      off = opaque_i(off - pl8);
      pe = e < n ? pe * r : r;
    }
  }
}

template <int MAXL>
__global__ void __launch_bounds__(kTriCols * kTriChunks, MAXL <= 16 ? 4 : 2) k_tri_b(float2* __restrict__ spec, int h, int w, int b,
                                                                 double w1, double w2, double w3,
                                                                 const double* __restrict__ mu_dev, double mu_host) {
  tri_b_body<MAXL>(blockIdx.x, gridDim.x, spec, h, w, b, w1, w2, w3, mu_dev, mu_host);
}

// ---------------------------------------------------------------------------
// Band DFT of real tensors along the bands, on the matrix cores.  With
// s = b/2 + 1 slices and the even / odd parts of A along the bands,
//   P_0 = A_0,  P_j = A_j + A_{b-j},  Q_0 = 0,  Q_j = A_j - A_{b-j}   (0 < j < s)
// (for even b, P_{b/2} = A_{b/2} and Q_{b/2} = 0: that row pairs with itself),
//   Re X_k =  sum_{j < s} P_j cos(2 pi j k / b),
//   Im X_k = -sum_{j < s} Q_j sin(2 pi j k / b),
// two real products of s x s terms, half the work of the full (2s x b)
// product.  Row 2k / 2k+1 of the output is the re / im plane of slice k: the
// planar slice layout [t][k][re|im][hw].
//
// A block (4 waves, v_mfma_f32_32x32x2f32) takes a 128-column strip of A;
// wave q forms both parts for its 32 columns and up to 96 slices at a time
// (three 32-row accumulators per part).  P and Q are formed as the strip is
// staged through LDS in chunks of 32 rows j; the cos / sin operands come
// from an LDS table of (2 pi m / b) as (cos, sin) pairs (one read for both
// products), their common index m = k j mod b advanced by 2k mod b per step.
constexpr int kDftRowTiles = 3;
constexpr int kDftCols = 128;   // strip width of both band transforms
struct DftSmem {
  // (cos, -sin)(2 pi m / b) (forward) or (cos, sin)(2 pi m / b) / b (inverse)
  // for m < b, and (0, 0) at m = b: the entry of the rows past the last slice
  float2 cs[LRSTV_MAX_SIDE_DEV + 1];
  union {
    struct {
      __align__(16) float p[kKC][kDftCols + 4], q[kKC][kDftCols + 4];
    };
    __align__(16) float et[2 * kKC][kDftCols + 4];   // inverse: E rows j, b - j of one 32-row block
  };
};

// Staging coordinates of a 32 x 128 chunk: thread t holds four columns of
// rows t / 32 + 8 e, e = 0..3.
LRSTV_DEV void dft_stage_coords(int t, int& sc, int& sr) {
  sc = 4 * (t & 31);
  sr = t >> 5;
}

// One pass over the rows k in [kb, kb + 32 NQ) of a 128-column strip (NQ
// row tiles: the passes of a short band axis take only the tiles that hold
// slices, and the contraction stops at the last row pair j < s).
template <int NQ>
LRSTV_DEV void band_dft_pass(DftSmem& sm, const float* __restrict__ src, float* __restrict__ dst, int kb, int s, int b,
                             int hw, int n0, int sc, int sr, int ncol, int wv, int li, int lk) {
  f32x16 are[NQ], aim[NQ];
  int idx[NQ], stp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int e = 0; e < 16; ++e) are[q][e] = aim[q][e] = 0.f;
    const int k = kb + 32 * q + li;
    // rows k >= s read the zero entry b, which the step b keeps in place
    idx[q] = k < s ? (k * lk) % b : b;   // j = lk at the first step
    stp[q] = k < s ? (2 * k) % b : b;
  }
  // rows j and b - j of the next chunk, four columns each
  float pa[4][4], pb[4][4];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = j0 + sr + 8 * e, jb = b - j;
      const bool pair = j > 0 && j < s && jb != j;
      load4(src + (int64_t)j * hw + n0 + sc, j < s ? ncol : 0, pa[e]);
      load4(src + (int64_t)(pair ? jb : 0) * hw + n0 + sc, pair ? ncol : 0, pb[e]);
    }
  };
  fetch(0);
  for (int j0 = 0; j0 < s; j0 += kKC) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float pv[4], qv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        pv[c] = pa[e][c] + pb[e][c];
        qv[c] = pa[e][c] - pb[e][c];
      }
      *reinterpret_cast<float4*>(&sm.p[sr + 8 * e][sc]) = make_float4(pv[0], pv[1], pv[2], pv[3]);
      *reinterpret_cast<float4*>(&sm.q[sr + 8 * e][sc]) = make_float4(qv[0], qv[1], qv[2], qv[3]);
    }
    __syncthreads();
    if (j0 + kKC < s) fetch(j0 + kKC);
    auto step = [&](int kk) {
      const float bp = sm.p[2 * kk + lk][32 * wv + li], bq = sm.q[2 * kk + lk][32 * wv + li];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float2 cs = sm.cs[idx[q]];
        are[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(cs.x, bp, are[q], 0, 0, 0);
        aim[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(cs.y, bq, aim[q], 0, 0, 0);
        idx[q] += stp[q];
        if (idx[q] >= b) idx[q] -= b;
      }
    };
    const int nkk = s - j0 < kKC ? (s - j0 + 1) >> 1 : kKC / 2;   // row pairs holding j < s
    int kk = 0;
    for (; kk + 4 <= nkk; kk += 4) {
      step(kk);
      step(kk + 1);
      step(kk + 2);
      step(kk + 3);
    }
    for (; kk < nkk; ++kk) step(kk);
    __syncthreads();
  }
  const int n = n0 + 32 * wv + li;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = kb + 32 * q + 8 * (e >> 2) + 4 * lk + (e & 3);
      if (k < s && n < hw) {
        dst[(int64_t)(2 * k) * hw + n] = are[q][e];
        dst[(int64_t)(2 * k + 1) * hw + n] = aim[q][e];
      }
    }
}

LRSTV_DEV void band_dft_body(int bid, int nblk, const float* __restrict__ A, int64_t a_stride, int n_t,
                             float* __restrict__ out, int hw, int b) {
  __shared__ DftSmem sm;
  for (int m = threadIdx.x; m <= b; m += blockDim.x) {
    double sv = 0.0, cv = 0.0;
    if (m < b) sincospi(2.0 * (double)m / (double)b, &sv, &cv);
    sm.cs[m] = make_float2((float)cv, (float)-sv);
  }
  __syncthreads();
  const int s = b / 2 + 1, M = 2 * s;
  const int TN = (hw + kDftCols - 1) / kDftCols, nstrips = n_t * TN;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 31, lk = lane >> 5;
  int sc, sr;
  dft_stage_coords(t, sc, sr);
  for (int strip = bid; strip < nstrips; strip += nblk) {
    const int tt = strip / TN, tn = strip - tt * TN, n0 = tn * kDftCols;
    const float* src = A + tt * a_stride;
    float* dst = out + (int64_t)tt * M * hw;
    const int ncol = hw - n0 - sc;   // columns of this thread's four that exist
    for (int kb = 0; kb < s; kb += 32 * kDftRowTiles) {
      const int nq = (s - kb + 31) >> 5;   // row tiles holding slices
      if (nq >= 3) band_dft_pass<3>(sm, src, dst, kb, s, b, hw, n0, sc, sr, ncol, wv, li, lk);
      else if (nq == 2) band_dft_pass<2>(sm, src, dst, kb, s, b, hw, n0, sc, sr, ncol, wv, li, lk);
      else band_dft_pass<1>(sm, src, dst, kb, s, b, hw, n0, sc, sr, ncol, wv, li, lk);
    }
  }
}

__global__ void __launch_bounds__(256, 2) k_band_dft(const float* __restrict__ A, int64_t a_stride, int n_t,
                                                  float* __restrict__ out, int hw, int b) {
  band_dft_body(blockIdx.x, gridDim.x, A, a_stride, n_t, out, hw, b);
}

// Inverse band DFT with Hermitian completion, as two real products over the
// s slices:
//   C_j = sum_{k < s} c_k Re X_k cos(2 pi j k / b) / b,
//   S_j = sum_{k < s} c_k Im X_k sin(2 pi j k / b) / b,   0 <= j < s,
//   E_j = C_j - S_j,   E_{b-j} = C_j + S_j   (0 < j, b - j != j),
// c_k = 1 for k = 0 and k = b/2, else 2 (slice k stands for k and b - k):
// cos and sin are even and odd in j around b, so that the s rows j give all
// b rows, at half the work of the full (b x 2s) product.
// Epilogue (optional): Gamma4 += mu (E - F) and FP64 partial sums of
// (E - F)^2, one fixed slot per block (grid = LRSTV_PARTS when part != NULL).
// Block shape as the forward transform: 128-column strips, wave q forms C and
// S for its 32 columns and up to 96 rows j at a time, so that both outputs
// E_j and E_{b-j} of an element come from one lane.  The outputs of each
// 32-row block go through LDS, so that the memory-bound epilogue (read F and
// Gamma4, write Gamma4 and E) runs on four-wide, row-contiguous accesses
// with four rows per thread in flight.
// One pass over the rows j in [jb, jb + 32 NQ) of a 128-column strip (as
// band_dft_pass: only the tiles holding rows j < s, the contraction up to
// the last slice pair); adds to the thread's FP64 partial of (E - F)^2.
template <int NQ>
LRSTV_DEV void band_idft_pass(DftSmem& sm, const float* __restrict__ src, float* __restrict__ dst,
                              const float* __restrict__ Ft, float* __restrict__ G4t, float mu, int jb, int s, int b,
                              int hw, int n0, int sc, int sr, int ncol, int wv, int li, int lk, double& acc) {
  f32x16 cc[NQ], ss[NQ];
  int idx[NQ], stp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int e = 0; e < 16; ++e) cc[q][e] = ss[q][e] = 0.f;
    const int j = jb + 32 * q + li;
    // rows j >= s read the zero entry b, which the step b keeps in place
    idx[q] = j < s ? (j * lk) % b : b;   // k = lk at the first step
    stp[q] = j < s ? (2 * j) % b : b;
  }
  // c_k Re X_k and c_k Im X_k of the next chunk of slices, four columns each
  float pr[4][4], pi[4][4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + sr + 8 * e;
      load4(src + (int64_t)(2 * k) * hw + n0 + sc, k < s ? ncol : 0, pr[e]);
      load4(src + (int64_t)(2 * k + 1) * hw + n0 + sc, k < s ? ncol : 0, pi[e]);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < s; k0 += kKC) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + sr + 8 * e;
      const float ck = (k == 0 || 2 * k == b) ? 1.f : 2.f;
      *reinterpret_cast<float4*>(&sm.p[sr + 8 * e][sc]) =
          make_float4(ck * pr[e][0], ck * pr[e][1], ck * pr[e][2], ck * pr[e][3]);
      *reinterpret_cast<float4*>(&sm.q[sr + 8 * e][sc]) =
          make_float4(ck * pi[e][0], ck * pi[e][1], ck * pi[e][2], ck * pi[e][3]);
    }
    __syncthreads();
    if (k0 + kKC < s) fetch(k0 + kKC);
    auto step = [&](int kk) {
      const float br = sm.p[2 * kk + lk][32 * wv + li], bi = sm.q[2 * kk + lk][32 * wv + li];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float2 cs = sm.cs[idx[q]];
        const float c = cs.x, sn = cs.y;
        cc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(c, br, cc[q], 0, 0, 0);
        ss[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(sn, bi, ss[q], 0, 0, 0);
        idx[q] += stp[q];
        if (idx[q] >= b) idx[q] -= b;
      }
    };
    const int nkk = s - k0 < kKC ? (s - k0 + 1) >> 1 : kKC / 2;   // row pairs holding k < s
    int kk = 0;
    for (; kk + 4 <= nkk; kk += 4) {
      step(kk);
      step(kk + 1);
      step(kk + 2);
      step(kk + 3);
    }
    for (; kk < nkk; ++kk) step(kk);
    __syncthreads();
  }
  // E_j = C_j - S_j (LDS row r) and E_{b-j} = C_j + S_j (row 32 + r) of
  // each 32-row block, then the epilogue over the block's rows
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (jb + 32 * q >= s) break;   // uniform
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = 8 * (e >> 2) + 4 * lk + (e & 3);
      sm.et[r][32 * wv + li] = cc[q][e] - ss[q][e];
      sm.et[32 + r][32 * wv + li] = cc[q][e] + ss[q][e];
    }
    __syncthreads();
#pragma unroll 4
    for (int u = 0; u < 8; ++u) {
      const int r = sr + 8 * u, j = jb + 32 * q + (r & 31);
      const bool lo_half = r < 32;
      if (j >= s || ncol <= 0 || (!lo_half && (j == 0 || b - j == j))) continue;
      const int64_t o = (int64_t)(lo_half ? j : b - j) * hw + n0 + sc;
      const float4 ev = *reinterpret_cast<const float4*>(&sm.et[r][sc]);
      const float e4[4] = {ev.x, ev.y, ev.z, ev.w};
      const int nv = ncol < 4 ? ncol : 4;
      if (nv == 4 && ((hw & 3) == 0)) {
        *reinterpret_cast<float4*>(dst + o) = ev;
        if (G4t) {
          const float4 f = *reinterpret_cast<const float4*>(Ft + o), g = *reinterpret_cast<const float4*>(G4t + o);
          const float f4[4] = {f.x, f.y, f.z, f.w};
          *reinterpret_cast<float4*>(G4t + o) =
              make_float4(g.x + mu * (e4[0] - f4[0]), g.y + mu * (e4[1] - f4[1]), g.z + mu * (e4[2] - f4[2]),
                          g.w + mu * (e4[3] - f4[3]));
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double dd = (double)e4[c] - (double)f4[c];
            acc += dd * dd;
          }
        }
      } else {
        for (int c = 0; c < nv; ++c) {
          dst[o + c] = e4[c];
          if (G4t) {
            const float f = Ft[o + c];
            G4t[o + c] = G4t[o + c] + mu * (e4[c] - f);
            const double dd = (double)e4[c] - (double)f;
            acc += dd * dd;
          }
        }
      }
    }
    __syncthreads();
  }
}

LRSTV_DEV void band_idft_body(int bid, int nblk, const float* __restrict__ X, int n_t, float* __restrict__ E,
                              int64_t e_stride, int hw, int b, const float* __restrict__ F, float* __restrict__ G4,
                              const double* __restrict__ mu_dev, double* __restrict__ part) {
  __shared__ DftSmem sm;
  __shared__ double red[4];
  for (int m = threadIdx.x; m <= b; m += blockDim.x) {
    double sv = 0.0, cv = 0.0;
    if (m < b) sincospi(2.0 * (double)m / (double)b, &sv, &cv);
    sm.cs[m] = make_float2((float)(cv * (1.0 / (double)b)), (float)(sv * (1.0 / (double)b)));
  }
  __syncthreads();
  const float mu = G4 ? (float)(*mu_dev) : 0.f;
  const int s = b / 2 + 1, K2 = 2 * s;
  const int TN = (hw + kDftCols - 1) / kDftCols, nstrips = n_t * TN;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 31, lk = lane >> 5;
  int sc, sr;
  dft_stage_coords(t, sc, sr);
  double acc = 0.0;   // per-thread partial of (E - F)^2 in FP64
  for (int strip = bid; strip < nstrips; strip += nblk) {
    const int tt = strip / TN, tn = strip - tt * TN, n0 = tn * kDftCols;
    const float* src = X + (int64_t)tt * K2 * hw;
    float* dst = E + tt * e_stride;
    const float* Ft = F ? F + tt * e_stride : nullptr;
    float* G4t = G4 ? G4 + tt * e_stride : nullptr;
    const int ncol = hw - n0 - sc;
    for (int jb = 0; jb < s; jb += 32 * kDftRowTiles) {
      const int nq = (s - jb + 31) >> 5;   // row tiles holding rows j < s
      if (nq >= 3) band_idft_pass<3>(sm, src, dst, Ft, G4t, mu, jb, s, b, hw, n0, sc, sr, ncol, wv, li, lk, acc);
      else if (nq == 2) band_idft_pass<2>(sm, src, dst, Ft, G4t, mu, jb, s, b, hw, n0, sc, sr, ncol, wv, li, lk, acc);
      else band_idft_pass<1>(sm, src, dst, Ft, G4t, mu, jb, s, b, hw, n0, sc, sr, ncol, wv, li, lk, acc);
    }
  }
  if (part) {
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) part[R_FRO_EF * LRSTV_PARTS + bid] = tot;
  }
}

__global__ void __launch_bounds__(256, 2) k_band_idft(const float* __restrict__ X, int n_t, float* __restrict__ E,
                                                   int64_t e_stride, int hw, int b, const float* __restrict__ F,
                                                   float* __restrict__ G4, const double* __restrict__ mu_dev,
                                                   double* __restrict__ part) {
  band_idft_body(blockIdx.x, gridDim.x, X, n_t, E, e_stride, hw, b, F, G4, mu_dev, part);
}

// ------------------------------------------------------------ launchers ---

// ------------------------------------------------------ batched phases ---
// All cubes of a packed ragged batch in one launch per phase.  Block b of the
// launch belongs to cube c with bt.bstart[c] <= b < bt.bstart[c + 1]; within
// the cube it runs as block b - bstart[c] of a grid of bstart[c+1] - bstart[c]
// blocks, the grid that cube would get alone (so its results, reductions
// included, do not depend on the other cubes).

__global__ void __launch_bounds__(256) k_rfft_w_batch(BatchTab bt, const float* __restrict__ T,
                                                      float2* __restrict__ spec) {
  extern __shared__ float2 sm[];
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (fft_h_reg_bit(g.w) != 0 || (g.mm & 2)) return;   // the register or DFT-matrix transform takes it
  rfft_w_body(q.bid, q.nblk, sm, T + g.off, spec + g.spec_off, g.h * g.b, g.w, g.nb_w);
}

__global__ void __launch_bounds__(kIrfftThreads) k_irfft_w_batch(BatchTab bt, const float2* __restrict__ spec,
                                                       float* __restrict__ Z, double* __restrict__ part) {
  extern __shared__ float2 sm[];
  const int c = blockIdx.x / LRSTV_PARTS;
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  if (fft_h_reg_bit(g.w) != 0 || (g.mm & 2)) return;   // the register or DFT-matrix transform takes it
  irfft_w_body(blockIdx.x - c * LRSTV_PARTS, LRSTV_PARTS, sm, spec + g.spec_off, Z + g.off, g.h * g.b, g.w, g.nb_wi,
               1.0f / ((float)g.h * (float)g.w), part ? part + (int64_t)c * R_COUNT * LRSTV_PARTS : nullptr);
}

__global__ void __launch_bounds__(kFftHThreads) k_fft_h_batch(BatchTab bt, float2* __restrict__ spec, int sign) {
  extern __shared__ float2 sm[];
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (fft_h_reg_bit(g.h) != 0 || (g.mm & 1)) return;   // the register or DFT-matrix transform takes it
  fft_h_body(q.bid, q.nblk, sm, spec + g.spec_off, g.h, g.w / 2 + 1, g.b, g.cw_h, sign);
}

template <int MAXL>
__global__ void __launch_bounds__(kTriCols * kTriChunks, MAXL <= 16 ? 4 : 2) k_tri_b_batch(BatchTab bt, float2* __restrict__ spec,
                                                                       double w1, double w2, double w3,
                                                                       const double* __restrict__ mu_dev) {
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  tri_b_body<MAXL>(q.bid, q.nblk, spec + g.spec_off, g.h, g.w, g.b, w1, w2, w3, mu_dev, 0.0);
}

// A: component stride a_stride from the cube's offset; slices at slice_base
__global__ void __launch_bounds__(256, 2) k_band_dft_batch(BatchTab bt, const float* __restrict__ A, int64_t a_stride,
                                                        float* __restrict__ slices) {
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  band_dft_body(q.bid, q.nblk, A + g.off, a_stride, 3, slices + g.slice_base, g.h * g.w, g.b);
}

__global__ void __launch_bounds__(256, 2) k_band_idft_batch(BatchTab bt, const float* __restrict__ slices,
                                                         float* __restrict__ E, int64_t e_stride,
                                                         const float* __restrict__ F, float* __restrict__ G4,
                                                         const double* __restrict__ mu_dev, double* __restrict__ part) {
  const int c = blockIdx.x / LRSTV_PARTS;
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  band_idft_body(blockIdx.x - c * LRSTV_PARTS, LRSTV_PARTS, slices + g.slice_base, 3, E + g.off, e_stride,
                 g.h * g.w, g.b, F + g.off, G4 + g.off, mu_dev, part + (int64_t)c * R_COUNT * LRSTV_PARTS);
}

static int rows_nb(int w) {
  int nb = 8;
  while (nb > 1 && (2 * nb + 1) * w * 8 > 48 * 1024) nb >>= 1;
  return nb;
}
// The inverse runs LRSTV_PARTS blocks of 512 threads per cube: up to 16 row
// pairs per pass (within 64 KB of LDS), so that a pass's butterflies reach
// most of the block's threads (1024 threads and 32 pairs left most of the
// blocks of a small cube idle: inverse w transforms of the ragged batch
// 0.40 -> 0.34 ms, of a 200 x 200 x 160 cube 60 -> 49 us).
static int rows_nb_inv(int w) {
  int nb = 16;
  while (nb > 1 && (2 * nb + 1) * w * 8 > 64 * 1024) nb >>= 1;
  return nb;
}

// Columns per block of the h FFT: 16 (whole 128-byte row segments) while the
// two LDS buffers and the twiddles stay within 80 KB (two blocks per CU).
static int fft_h_stride(int h) { return h + (((2 - h) % 32) + 32) % 32; }
static size_t fft_h_lds_bytes(int h, int cw) { return ((size_t)2 * cw * fft_h_stride(h) + h) * sizeof(float2); }
static int cols_cw(int h) {
  int cw = 16;
  while (cw > 1 && fft_h_lds_bytes(h, cw) > 80 * 1024) cw >>= 1;
  return cw;
}

template <int P, int Q>
__global__ void __launch_bounds__(kRfftPairs * kPairThreads) k_rfft_w_reg(const float* __restrict__ T,
                                                                       float2* __restrict__ spec, int nrows) {
  rfft_w_reg_body<P, Q, kRfftPairs>(blockIdx.x, gridDim.x, T, spec, nrows);
}
template <int P, int Q>
__global__ void __launch_bounds__(kRfftPairs * kPairThreads) k_rfft_w_reg_batch(BatchTab bt, const float* __restrict__ T,
                                                                             float2* __restrict__ spec) {
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (g.w != P * Q) return;   // another length (or the Stockham path) takes that cube
  rfft_w_reg_body<P, Q, kRfftPairs>(q.bid, q.nblk, T + g.off, spec + g.spec_off, g.h * g.b);
}
template <int P, int Q>
__global__ void __launch_bounds__(kIrfftPairs * kPairThreads) k_irfft_w_reg(const float2* __restrict__ spec,
                                                                         float* __restrict__ Z, int nrows, float scale,
                                                                         double* __restrict__ part) {
  irfft_w_reg_body<P, Q, kIrfftPairs>(blockIdx.x, gridDim.x, spec, Z, nrows, scale, part);
}
template <int P, int Q>
__global__ void __launch_bounds__(kIrfftPairs * kPairThreads) k_irfft_w_reg_batch(BatchTab bt,
                                                                               const float2* __restrict__ spec,
                                                                               float* __restrict__ Z,
                                                                               double* __restrict__ part) {
  const int c = blockIdx.x / LRSTV_PARTS;
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  if (g.w != P * Q) return;
  irfft_w_reg_body<P, Q, kIrfftPairs>(blockIdx.x - c * LRSTV_PARTS, LRSTV_PARTS, spec + g.spec_off, Z + g.off,
                                      g.h * g.b, 1.0f / ((float)g.h * (float)g.w),
                                      part ? part + (int64_t)c * R_COUNT * LRSTV_PARTS : nullptr);
}

// The register w transforms for w = 64, 128, 256 (false for other widths).
// Single cube when bt is null, else every cube of that width in the batch.
static bool launch_rfft_w_reg(const float* T, float2* spec, int w, int nrows, const BatchTab* bt, hipStream_t s) {
#define LRSTV_RFFT_REG(P, Q)                                                                                    \
  if (w == P * Q) {                                                                                             \
    if (bt) {                                                                                                   \
      hipLaunchKernelGGL((k_rfft_w_reg_batch<P, Q>), dim3(bt->nblocks), dim3(kRfftPairs * kPairThreads), 0, s, *bt, \
                         T, spec);                                                                              \
    } else {                                                                                                    \
      const int npairs = (nrows + 1) / 2, g = (npairs + kRfftPairs - 1) / kRfftPairs;                           \
      hipLaunchKernelGGL((k_rfft_w_reg<P, Q>), dim3(g < 4096 ? g : 4096), dim3(kRfftPairs * kPairThreads), 0, s, T, \
                         spec, nrows);                                                                          \
    }                                                                                                           \
    return true;                                                                                                \
  }
  LRSTV_RFFT_REG(16, 16)
  LRSTV_RFFT_REG(16, 8)
  LRSTV_RFFT_REG(8, 8)
#undef LRSTV_RFFT_REG
  return false;
}
static bool launch_irfft_w_reg(const float2* spec, float* Z, int w, int nrows, float scale, double* part,
                               const BatchTab* bt, hipStream_t s) {
#define LRSTV_IRFFT_REG(P, Q)                                                                                      \
  if (w == P * Q) {                                                                                                \
    if (bt)                                                                                                        \
      hipLaunchKernelGGL((k_irfft_w_reg_batch<P, Q>), dim3(bt->nc * LRSTV_PARTS), dim3(kIrfftPairs * kPairThreads), 0, \
                         s, *bt, spec, Z, part);                                                                   \
    else                                                                                                           \
      hipLaunchKernelGGL((k_irfft_w_reg<P, Q>), dim3(LRSTV_PARTS), dim3(kIrfftPairs * kPairThreads), 0, s, spec, Z,  \
                         nrows, scale, part);                                                                      \
    return true;                                                                                                   \
  }
  LRSTV_IRFFT_REG(16, 16)
  LRSTV_IRFFT_REG(16, 8)
  LRSTV_IRFFT_REG(8, 8)
#undef LRSTV_IRFFT_REG
  return false;
}

void launch_rfft_w(const float* T, float2* spec, int h, int w, int b, hipStream_t s) {
  if (dft_mm_len(w, kMmMaxW)) {
    launch_dftmm_rw(T, spec, h, w, b, s);
    return;
  }
  if (launch_rfft_w_reg(T, spec, w, h * b, nullptr, s)) return;
  const int nrows = h * b, nb = rows_nb(w);
  const size_t lds = (size_t)(2 * nb + 1) * w * sizeof(float2);
  int grid = (nrows + 2 * nb - 1) / (2 * nb);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_rfft_w, dim3(grid), dim3(256), lds, s, T, spec, nrows, w, nb);
}

void launch_irfft_w(const float2* spec, float* Z, int h, int w, int b, double* part, hipStream_t s) {
  if (dft_mm_len(w, kMmMaxW)) {
    launch_dftmm_irw(spec, Z, h, w, b, part, s);
    return;
  }
  const int nrows = h * b, nb = rows_nb_inv(w);
  const size_t lds = (size_t)(2 * nb + 1) * w * sizeof(float2);
  const float scale = 1.0f / ((float)h * (float)w);
  if (launch_irfft_w_reg(spec, Z, w, nrows, scale, part, nullptr, s)) return;
  hipLaunchKernelGGL(k_irfft_w, dim3(LRSTV_PARTS), dim3(kIrfftThreads), lds, s, spec, Z, nrows, w, nb, scale, part);
}


template <int P, int Q, int S>
__global__ void __launch_bounds__(kFftRegCols * (P > Q ? P : Q)) k_fft_h_reg_batch(BatchTab bt, float2* __restrict__ spec) {
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (g.h != P * Q) return;   // another length (or the Stockham path) takes that cube
  fft_h_reg_body<P, Q, S>(q.bid, q.nblk, spec + g.spec_off, g.w / 2 + 1, g.b);
}

// Launches the register FFT when h is one of its lengths; false otherwise.
template <int S>
static bool launch_fft_h_reg(float2* spec, int h, int wc, int b, int grid, const BatchTab* bt, hipStream_t s) {
#define LRSTV_FFT_REG(P, Q)                                                                                   \
  if (h == P * Q) {                                                                                           \
    if (bt)                                                                                                   \
      hipLaunchKernelGGL((k_fft_h_reg_batch<P, Q, S>), dim3(bt->nblocks), dim3(fft_reg_threads<P, Q>()), 0, s, \
                         *bt, spec);                                                                          \
    else                                                                                                      \
      hipLaunchKernelGGL((k_fft_h_reg<P, Q, S>), dim3(grid), dim3(fft_reg_threads<P, Q>()), 0, s, spec, wc, b); \
    return true;                                                                                              \
  }
  LRSTV_FFT_REG(16, 16)
  LRSTV_FFT_REG(16, 8)
  LRSTV_FFT_REG(8, 8)
#undef LRSTV_FFT_REG
  return false;
}

// Dynamic LDS above the 64 KB default is granted once per process (before any
// capture: the handle's set-up and the stand-alone Z-solve call this).
static size_t g_fft_h_granted = 65536;
void prepare_fft_h(size_t lds) {
  if (lds <= g_fft_h_granted) return;
  if (hipFuncSetAttribute((const void*)k_fft_h, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess &&
      hipFuncSetAttribute((const void*)k_fft_h_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
          hipSuccess)
    g_fft_h_granted = lds;
}

void launch_fft_h(float2* spec, int h, int w, int b, int sign, hipStream_t s) {
  if (dft_mm_len(h, kMmMaxH)) {
    launch_dftmm_h(spec, h, w, b, sign, s);
    return;
  }
  const int wc = w / 2 + 1;
  const int cw = fft_h_reg_bit(h) ? kFftRegCols : cols_cw(h);
  const int64_t g = ((int64_t)b * wc + cw - 1) / cw;
  const int grid = (int)(g < 8192 ? g : 8192);
  if (sign < 0 ? launch_fft_h_reg<-1>(spec, h, wc, b, grid, nullptr, s) : launch_fft_h_reg<1>(spec, h, wc, b, grid, nullptr, s))
    return;
  prepare_fft_h(fft_h_lds_bytes(h, cw));
  hipLaunchKernelGGL(k_fft_h, dim3(grid), dim3(kFftHThreads), fft_h_lds_bytes(h, cw), s, spec, h, wc, b, cw, sign);
}

// Register chunk length of the band solve: L = ceil(b / kTriChunks) <= 16
// for b <= 256, else <= 32 (LRSTV_MAX_SIDE = 512).
static int tri_groups(int h, int w) {
  const int64_t g = ((int64_t)h * (w / 2 + 1) + kTriCols - 1) / kTriCols;
  return (int)(g < 16384 ? g : 16384);
}

void launch_tri_b(float2* spec, int h, int w, int b, const double wts[3], const double* mu, double mu_host,
                  hipStream_t s) {
  const int grid = tri_groups(h, w);
  if ((b + kTriChunks - 1) / kTriChunks <= 16)
    hipLaunchKernelGGL(k_tri_b<16>, dim3(grid), dim3(kTriCols * kTriChunks), 0, s, spec, h, w, b, wts[0], wts[1],
                       wts[2], mu, mu_host);
  else
    hipLaunchKernelGGL(k_tri_b<32>, dim3(grid), dim3(kTriCols * kTriChunks), 0, s, spec, h, w, b, wts[0], wts[1],
                       wts[2], mu, mu_host);
}

static int dft_tile(int b) {
  int P = 64;
  while (P > 16 && ((size_t)2 * b + (size_t)b * P) * 4 > 60 * 1024) P >>= 1;
  return P;
}

void launch_band_dft(const float* A, int64_t a_stride, int n_t, float* slices, int h, int w, int b, hipStream_t s) {
  const int hw = h * w;
  const int64_t nstrips = (int64_t)n_t * ((hw + kDftCols - 1) / kDftCols);
  const int grid = (int)(nstrips < 512 ? nstrips : 512);
  hipLaunchKernelGGL(k_band_dft, dim3(grid), dim3(256), 0, s, A, a_stride, n_t, slices, hw, b);
}

void launch_band_idft(const float* slices, int n_t, float* E, int64_t e_stride, int h, int w, int b,
                      const float* F, float* G4, const double* mu, double* part, hipStream_t s) {
  const int hw = h * w;
  const int64_t nstrips = (int64_t)n_t * ((hw + kDftCols - 1) / kDftCols);
  const int grid = part ? LRSTV_PARTS : (int)(nstrips < 2048 ? nstrips : 2048);
  hipLaunchKernelGGL(k_band_idft, dim3(grid), dim3(256), 0, s, slices, n_t, E, e_stride, hw, b, F, G4, mu, part);
}

// ---------------------------------------------------- batched launchers ---
// Per-cube block counts of each phase (host), the same as the single-cube
// launchers would use.
int phase_blocks(int phase, int h, int w, int b) {
  const int64_t N = (int64_t)h * w * b;
  const int wc = w / 2 + 1;
  switch (phase) {
    case PH_LRHS: {
      // one element per thread up to 16.7 M voxels: more loads in flight than
      // a grid-stride loop over fewer blocks (8192 blocks took 0.147 ms at
      // 256 x 256 x 191, 48,896 take 0.132)
      const int64_t g = (N + 255) / 256;
      return (int)(g < 65536 ? g : 65536);
    }
    case PH_RFFT_W: {
      if (dft_mm_len(w, kMmMaxW)) return dftmm_blocks_w(h, w, b);
      const int nb = rows_nb(w);
      const int64_t g = ((int64_t)h * b + 2 * nb - 1) / (2 * nb);
      return (int)(g < 4096 ? g : 4096);
    }
    case PH_FFT_H: {
      if (dft_mm_len(h, kMmMaxH)) return dftmm_blocks_h(h, w, b);
      const int cw = fft_h_reg_bit(h) ? kFftRegCols : cols_cw(h);
      const int64_t g = ((int64_t)b * wc + cw - 1) / cw;
      return (int)(g < 8192 ? g : 8192);
    }
    case PH_TRI_B: return tri_groups(h, w);
    case PH_BAND_DFT: {
      // two blocks per CU (register budget): the strips of a 256 x 256 cube
      // in one round of 512 blocks
      const int64_t t = (int64_t)3 * (((int64_t)h * w + kDftCols - 1) / kDftCols);
      return (int)(t < 512 ? t : 512);
    }
    default: return LRSTV_PARTS;
  }
}

int geo_rows_nb(int w) { return rows_nb(w); }
int geo_rows_nb_inv(int w) { return rows_nb_inv(w); }
int geo_cols_cw(int h) { return cols_cw(h); }
size_t geo_fft_h_lds(int h) { return fft_h_lds_bytes(h, cols_cw(h)); }

// As for the h transform, every cube takes the path of its own w.
void launch_rfft_w_batch(const BatchTab& bt, const float* T, float2* spec, hipStream_t s) {
  for (int w : {64, 128, 256})
    if (bt.reg_w_mask & fft_h_reg_bit(w)) launch_rfft_w_reg(T, spec, w, 0, &bt, s);
  if (bt.stockham_w) hipLaunchKernelGGL(k_rfft_w_batch, dim3(bt.nblocks), dim3(256), bt.lds_w, s, bt, T, spec);
  if (bt.mm_w) launch_dftmm_rw_batch(bt, T, spec, s);
}

void launch_irfft_w_batch(const BatchTab& bt, const float2* spec, float* Z, double* part, hipStream_t s) {
  for (int w : {64, 128, 256})
    if (bt.reg_w_mask & fft_h_reg_bit(w)) launch_irfft_w_reg(spec, Z, w, 0, 0.f, part, &bt, s);
  if (bt.stockham_w)
    hipLaunchKernelGGL(k_irfft_w_batch, dim3(bt.nc * LRSTV_PARTS), dim3(kIrfftThreads), bt.lds_wi, s, bt, spec, Z,
                       part);
  if (bt.mm_w) launch_dftmm_irw_batch(bt, spec, Z, part, s);
}

void launch_fft_h_batch(const BatchTab& bt, float2* spec, int sign, hipStream_t s) {
  // every cube takes the path of its own h (as it would alone): one launch
  // per register length present, one Stockham launch for the other cubes
  for (int h : {64, 128, 256})
    if (bt.reg_h_mask & fft_h_reg_bit(h)) {
      if (sign < 0) launch_fft_h_reg<-1>(spec, h, 0, 0, 0, &bt, s);
      else launch_fft_h_reg<1>(spec, h, 0, 0, 0, &bt, s);
    }
  if (bt.stockham_h)
    hipLaunchKernelGGL(k_fft_h_batch, dim3(bt.nblocks), dim3(kFftHThreads), bt.lds_h, s, bt, spec, sign);
  if (bt.mm_h) launch_dftmm_h_batch(bt, spec, sign, s);
}

void launch_tri_b_batch(const BatchTab& bt, float2* spec, const double wts[3], const double* mu, hipStream_t s) {
  if (bt.max_b <= 16 * kTriChunks)
    hipLaunchKernelGGL(k_tri_b_batch<16>, dim3(bt.nblocks), dim3(kTriCols * kTriChunks), 0, s, bt, spec, wts[0],
                       wts[1], wts[2], mu);
  else
    hipLaunchKernelGGL(k_tri_b_batch<32>, dim3(bt.nblocks), dim3(kTriCols * kTriChunks), 0, s, bt, spec, wts[0],
                       wts[1], wts[2], mu);
}

void launch_band_dft_batch(const BatchTab& bt, const float* A, int64_t a_stride, float* slices, hipStream_t s) {
  hipLaunchKernelGGL(k_band_dft_batch, dim3(bt.nblocks), dim3(256), 0, s, bt, A, a_stride, slices);
}

void launch_band_idft_batch(const BatchTab& bt, const float* slices, float* E, int64_t e_stride, const float* F,
                            float* G4, const double* mu, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_band_idft_batch, dim3(bt.nc * LRSTV_PARTS), dim3(256), 0, s, bt, slices, E, e_stride, F,
                     G4, mu, part);
}

}  // namespace lrstv
