// Element-wise and stencil kernels of one ADMM iteration (Sec. III-C):
//   k_lrhs        L-update (1st step, full Tucker rank) fused with the
//                 right-hand side T_z of the Z-update (adjoint differences);
//   k_grad_shrink forward differences D_w Z, F-update (soft-threshold),
//                 Gamma3 / Gamma2 ascent, S-update and Gamma1 ascent, and the
//                 t-SVT input A = F - Gamma4/mu; Frobenius / max residuals;
//   k_fill, k_init_state, k_finish_iter, k_mu_step: state set-up,
//                 fixed-order FP64 residual reduction and the penalty update.
//
// Cubes are FP32 [b][h][w] (w fastest); differences are periodic.  The
// gradient-shaped variables F, E, Gamma3, Gamma4 are three cubes spaced by
// `ts` floats.  mu lives on the device so that iterations can be replayed
// without host involvement.
#include "common.hpp"
#include "kernels.hpp"

namespace lrstv {

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// p[i] = a value in [-1, 1) from a 32-bit integer hash of (i, seed)
// (lowbias32 mixing), for timing runs on data that is not all zeros.
__global__ void k_fill_hash(float* __restrict__ p, int64_t n, uint32_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[i] = (float)(x >> 8) * (2.0f / 16777216.0f) - 1.0f;
  }
}

__global__ void k_set_mu(double* mu, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *mu = v;
}

// L = 1/2 (O - S - N + Z + (Gamma1 - Gamma2)/mu)   (N = 0 without the noise term)
// T_z = mu L + Gamma2 + sum_n w_n D_n^T (mu F_n - Gamma3_n),
// (D_n^T y)[v] = y[v - e_n] - y[v].
LRSTV_DEV void lrhs_body(int bid, int nblk, const float* __restrict__ O, const float* __restrict__ S,
                         const float* __restrict__ Nz, const float* __restrict__ Z, const float* __restrict__ G1, const float* __restrict__ G2,
                         const float* __restrict__ F, const float* __restrict__ G3, int64_t ts,
                         float* __restrict__ L, float* __restrict__ Tz, int h, int w, int b, float w1, float w2,
                         float w3, const double* __restrict__ mu_dev) {
  const int64_t hw = (int64_t)h * w, N = hw * b;
  const double mud = *mu_dev;
  const float mu = (float)mud, imu = (float)(1.0 / mud);
  for (int64_t q = bid * (int64_t)blockDim.x + threadIdx.x; q < N; q += (int64_t)nblk * blockDim.x) {
    const int x = (int)(q % w);
    const int i = (int)((q / w) % h);
    const int j = (int)(q / hw);
    const float nq = Nz ? Nz[q] : 0.f;
    const float l = 0.5f * (O[q] - S[q] - nq + Z[q] + (G1[q] - G2[q]) * imu);
    L[q] = l;
    const int64_t qh = (i == 0) ? q + (int64_t)(h - 1) * w : q - w;
    const int64_t qw = (x == 0) ? q + (w - 1) : q - 1;
    const int64_t qb = (j == 0) ? q + (int64_t)(b - 1) * hw : q - hw;
    const float* F1 = F + ts;
    const float* F2 = F + 2 * ts;
    const float* H1 = G3 + ts;
    const float* H2 = G3 + 2 * ts;
    const float y0 = mu * F[q] - G3[q], y0n = mu * F[qh] - G3[qh];
    const float y1 = mu * F1[q] - H1[q], y1n = mu * F1[qw] - H1[qw];
    const float y2 = mu * F2[q] - H2[q], y2n = mu * F2[qb] - H2[qb];
    Tz[q] = mu * l + G2[q] + w1 * (y0n - y0) + w2 * (y1n - y1) + w3 * (y2n - y2);
  }
}


// All cubes of a packed batch in one launch: block ranges per cube from
// bt.bstart (each cube keeps the block count it would have alone).
__global__ void __launch_bounds__(256) k_lrhs_batch(BatchTab bt, BatchPtrs p, float w1, float w2, float w3,
                                                    const double* __restrict__ mu_dev) {
  const int c = find_cube(bt.bstart, bt.nc, blockIdx.x);
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  const int64_t o = g.off;
  lrhs_body(blockIdx.x - bt.bstart[c], bt.bstart[c + 1] - bt.bstart[c], p.O + o, p.S + o,
            p.N ? p.N + o : nullptr, p.Z + o, p.G1 + o,
            p.G2 + o, p.F + o, p.G3 + o, p.ts, p.L + o, p.T + o, g.h, g.w, g.b, w1, w2, w3, mu_dev);
}

// G_n = w_n D_n Z (forward, periodic)
// F_n = R_{tau/mu}( 1/2 (G_n + Gamma3_n/mu + E_n + Gamma4_n/mu) )
//   (isotropic: U_n = 1/2 (...), F = max(1 - (tau/mu) / ||U||_2, 0) U with
//    the norm over the three directions of the voxel)
// Gamma3_n += mu (G_n - F_n);   A_n = F_n - Gamma4_n / mu
// Gamma2 += mu (L - Z)
// S = R_{lambda/mu}(O - L - N + Gamma1/mu);   with the noise term
// N' = (mu (O - L - S) + Gamma1) / (mu + 2 beta);   Gamma1 += mu (O - L - S - N')
// Residual partials (one per block, fixed grid of LRSTV_PARTS blocks):
//   max|O-L-S|, max|L-Z|, sum (O-L-S)^2, sum (L-Z)^2, sum_n (G_n - F_n)^2.
LRSTV_DEV void grad_shrink_body(
    int bid, const float* __restrict__ O, const float* __restrict__ L, const float* __restrict__ Z,
    float* __restrict__ S, float* __restrict__ Nz, float* __restrict__ G1, float* __restrict__ G2,
    float* __restrict__ F,
    const float* __restrict__ E, float* __restrict__ G3, const float* __restrict__ G4, float* __restrict__ A,
    int64_t ts, int64_t as, int h, int w, int b, float w1, float w2, float w3, float tau, float lam, int iso,
    double beta, const double* __restrict__ mu_dev,
    double* __restrict__ part /* [R_COUNT][LRSTV_PARTS] of this cube */) {
  constexpr int nblk = LRSTV_PARTS;
  __shared__ double red[8];
  const int64_t hw = (int64_t)h * w, N = hw * b;
  const double mud = *mu_dev;
  const float mu = (float)mud, imu = (float)(1.0 / mud);
  const float tmu = (float)(tau / mud), lmu = (float)(lam / mud);
  const float inb = (float)(1.0 / (mud + 2.0 * beta));   // the noise step's divisor
  const float wn[3] = {w1, w2, w3};
  // maxima in FP32 (exact), sums of squares in FP64 from the first term on
  float m_ols = 0.f, m_lz = 0.f;
  double s_ols = 0.0, s_lz = 0.0, s_dzf = 0.0;
  // (x, i, j) of q advanced incrementally by the grid stride (no divisions
  // per element): stride = dz h w + dy w + dx with dx < w, dy < h
  const int64_t q0 = bid * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)nblk * blockDim.x;
  const int dx = (int)(stride % w), dy = (int)((stride / w) % h), dz = (int)(stride / hw);
  int x = (int)(q0 % w), i = (int)((q0 / w) % h), j = (int)(q0 / hw);
  for (int64_t q = q0; q < N; q += stride) {
    const float z = Z[q], l = L[q], o = O[q];
    const int64_t qn[3] = {(i == h - 1) ? q - (int64_t)(h - 1) * w : q + w, (x == w - 1) ? q - (w - 1) : q + 1,
                           (j == b - 1) ? q - (int64_t)(b - 1) * hw : q + hw};
    float gv[3], g3v[3], g4v[3], uv[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t o3 = n * ts + q;
      gv[n] = wn[n] * (Z[qn[n]] - z);
      g3v[n] = G3[o3];
      g4v[n] = G4[o3];
      uv[n] = 0.5f * (gv[n] + g3v[n] * imu + E[o3] + g4v[n] * imu);
    }
    float gscale = 0.f;   // isotropic: the common factor of the voxel's three components
    if (iso) {
      const float nrm = sqrtf(uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2]);
      gscale = nrm > tmu ? 1.0f - tmu / nrm : 0.f;
    }
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t o3 = n * ts + q;
      const float g = gv[n], g3 = g3v[n], g4 = g4v[n];
      const float f = iso ? uv[n] * gscale : soft_threshold(uv[n], tmu);
      F[o3] = f;
      G3[o3] = g3 + mu * (g - f);
      A[n * as + q] = f - g4 * imu;
      const double d = (double)g - (double)f;
      s_dzf += d * d;
    }
    G2[q] = G2[q] + mu * (l - z);
    const float g1 = G1[q];
    const float nold = Nz ? Nz[q] : 0.f;
    const float s = soft_threshold(o - l - nold + g1 * imu, lmu);
    S[q] = s;
    float nn = 0.f;
    if (Nz) {
      nn = (mu * (o - l - s) + g1) * inb;
      Nz[q] = nn;
    }
    const float r = o - l - s - nn, dz2 = l - z;
    G1[q] = g1 + mu * r;
    m_ols = fmaxf(m_ols, fabsf(r));
    m_lz = fmaxf(m_lz, fabsf(dz2));
    s_ols += (double)r * (double)r;
    s_lz += (double)dz2 * (double)dz2;
    x += dx;
    if (x >= w) { x -= w; ++i; }
    i += dy;
    if (i >= h) { i -= h; ++j; }
    j += dz;
  }
  const double bm_ols = block_max((double)m_ols, red);
  const double bm_lz = block_max((double)m_lz, red);
  const double bs_ols = block_sum(s_ols, red);
  const double bs_lz = block_sum(s_lz, red);
  const double bs_dzf = block_sum(s_dzf, red);
  if (threadIdx.x == 0) {
    part[R_INF_OLS * LRSTV_PARTS + bid] = bm_ols;
    part[R_INF_LZ * LRSTV_PARTS + bid] = bm_lz;
    part[R_FRO_OLS * LRSTV_PARTS + bid] = bs_ols;
    part[R_FRO_LZ * LRSTV_PARTS + bid] = bs_lz;
    part[R_FRO_DZF * LRSTV_PARTS + bid] = bs_dzf;
  }
}


// Batch: LRSTV_PARTS blocks per cube, cube c's residual slots at part + c R_COUNT LRSTV_PARTS.
__global__ void __launch_bounds__(512) k_grad_shrink_batch(BatchTab bt, BatchPtrs p, float w1, float w2, float w3,
                                                           float tau, float lam, int iso, double beta,
                                                           const double* __restrict__ mu_dev,
                                                           double* __restrict__ part) {
  const int c = blockIdx.x / LRSTV_PARTS;
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  const int64_t o = g.off;
  grad_shrink_body(blockIdx.x - c * LRSTV_PARTS, p.O + o, p.L + o, p.Z + o, p.S + o, p.N ? p.N + o : nullptr,
                   p.G1 + o, p.G2 + o, p.F + o,
                   p.E + o, p.G3 + o, p.G4 + o, p.A + o, p.ts, p.ts, g.h, g.w, g.b, w1, w2, w3, tau, lam, iso, beta,
                   mu_dev,
                   part + (int64_t)c * R_COUNT * LRSTV_PARTS);
}

// One block per cube: fixed-order reduction of the residual partials.
// out[cube][R_COUNT] (and optionally res_user[cube][R_COUNT]); sets *flag to
// 1 when a residual is not finite.  With a stopping state (halt != NULL): a
// halted cube is skipped (its residuals stay those of its last iteration);
// otherwise the cube's iteration count is advanced, *ran is set, and the
// cube halts when max(||O - L - S||_inf, ||L - Z||_inf) <= eps (eps > 0),
// Algorithm 1's convergence check.
__global__ void k_finish_iter(const double* __restrict__ part, int n_cubes, const double* __restrict__ mu_dev,
                              double* __restrict__ out, double* __restrict__ res_user, int* __restrict__ flag,
                              int* __restrict__ halt, int* __restrict__ iters, int* __restrict__ ran,
                              const double* __restrict__ eps_dev) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  if (c >= n_cubes) return;
  if (halt && halt[c]) return;
  const double* p = part + (int64_t)c * R_COUNT * LRSTV_PARTS;
  double v[R_COUNT];
  double nbad = 0.0;
  for (int r = 0; r < R_COUNT; ++r) {
    double a = 0.0;
    const bool is_max = (r == R_INF_OLS || r == R_INF_LZ);
    for (int k = threadIdx.x; k < LRSTV_PARTS; k += blockDim.x) {
      const double x = p[r * LRSTV_PARTS + k];
      if (!isfinite(x)) nbad += 1.0;
      else a = is_max ? fmax(a, x) : a + x;
    }
    v[r] = is_max ? block_max(a, red) : block_sum(a, red);
  }
  nbad = block_sum(nbad, red);
  if (threadIdx.x == 0) {
    const double mu = *mu_dev;
    double o[R_COUNT];
    o[R_INF_OLS] = v[R_INF_OLS];
    o[R_INF_LZ] = v[R_INF_LZ];
    o[R_FRO_OLS] = sqrt(v[R_FRO_OLS]);
    o[R_FRO_LZ] = sqrt(v[R_FRO_LZ]);
    o[R_FRO_DZF] = sqrt(v[R_FRO_DZF]);
    o[R_FRO_EF] = sqrt(v[R_FRO_EF]);
    o[R_DUAL_Z] = mu * sqrt(v[R_DUAL_Z]);
    bool bad = nbad > 0.0;
    for (int r = 0; r < R_COUNT; ++r) {
      if (nbad > 0.0) o[r] = __longlong_as_double(0x7ff8000000000000ULL);  // NaN
      out[c * R_COUNT + r] = o[r];
      if (res_user) res_user[c * R_COUNT + r] = o[r];
      bad |= !isfinite(o[r]);
    }
    if (bad) atomicExch(flag, 1);
    if (halt) {
      iters[c] += 1;
      *ran = 1;
      const double eps = *eps_dev;
      if (eps > 0.0 && fmax(o[R_INF_OLS], o[R_INF_LZ]) <= eps) halt[c] = 1;
    }
  }
}

// mu <- min(rho mu, mu_max) (7th step).  With a stopping state the step is
// taken only when some cube ran this iteration, and the marker is cleared.
__global__ void k_mu_step(double* mu, double rho, double mu_max, int* __restrict__ ran) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (!ran || *ran) *mu = fmin(rho * *mu, mu_max);
    if (ran) *ran = 0;
  }
}

__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_set_double(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ------------------------------------------------------------ launchers ---

void launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, p, n, v);
}

void launch_copy(float* dst, const float* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, dst, src, n);
}

void launch_fill_hash(float* p, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_fill_hash, dim3(grid), dim3(256), 0, s, p, n, seed);
}

void launch_set_mu(double* mu, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_mu, dim3(1), dim3(64), 0, s, mu, v);
}



void launch_finish_iter(const double* part, int n_cubes, const double* mu, double* out, double* res_user,
                        int* flag, const StopState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_iter, dim3(n_cubes), dim3(256), 0, s, part, n_cubes, mu, out, res_user, flag,
                     st ? st->halt : nullptr, st ? st->iters : nullptr, st ? st->ran : nullptr,
                     st ? st->eps : nullptr);
}

void launch_mu_step(double* mu, double rho, double mu_max, int* ran, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_step, dim3(1), dim3(64), 0, s, mu, rho, mu_max, ran);
}

void launch_fill_int(int* p, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_fill_int, dim3(grid), dim3(256), 0, s, p, n, v);
}

void launch_set_double(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, s, p, v);
}

void launch_lrhs_batch(const BatchTab& bt, const BatchPtrs& p, const Weights& wt, const double* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_lrhs_batch, dim3(bt.nblocks), dim3(256), 0, s, bt, p, (float)wt.w[0], (float)wt.w[1],
                     (float)wt.w[2], mu);
}

void launch_grad_shrink_batch(const BatchTab& bt, const BatchPtrs& p, const Weights& wt, const double* mu,
                              double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_shrink_batch, dim3(bt.nc * LRSTV_PARTS), dim3(512), 0, s, bt, p, (float)wt.w[0],
                     (float)wt.w[1], (float)wt.w[2], (float)wt.tau, (float)wt.lam, wt.iso, wt.beta, mu, part);
}

}  // namespace lrstv
