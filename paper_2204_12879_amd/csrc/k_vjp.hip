// Element-wise and stencil kernels of the adjoint (vector-Jacobian product)
// of one ADMM iteration (Sec. III-C, Algorithm 1, taken in reverse).
//
// Notation: x' is a variable after the iteration, gx the cotangent of x
// (ga.* the given cotangents of the new state, gb.* those of the old state
// that are produced), mu the penalty of the iteration.  The shrink masks and
// signs are read from the iteration's own outputs: R_d(u) != 0 exactly when
// |u| > d, with the sign of u.
//
//   k_vjp_post    multiplier ascents (6th step) and S-update (5th step):
//                 gL, gZ' partial, gF' partial, the t-SVT direction gE' and
//                 point A = F' - Gamma4/mu, lambda partials
//   k_vjp_shrinkf t-SVT cotangent into F' and Gamma4, F-update (3rd step)
//                 shrink, tau partials, gG_n = mu ga.Gamma3_n + gU_n / 2
//   k_vjp_divt    gZ' = gZ' partial + sum_n w_n D_n^T gG_n
//   (Z-solve)     gT = (mu (I + D_w^* D_w))^-1 gZ'  (symmetric operator)
//   k_vjp_pre     right-hand side and L-update (2nd and 1st steps)
//   k_vjp_finish  fixed-order FP64 sums of the parameter cotangents
#include "common.hpp"
#include "kernels.hpp"

namespace lrstv {

// ga.* may be NULL as a whole (zero cotangent of the new state)
__global__ void __launch_bounds__(256) k_vjp_post(VjpCube c, const double* __restrict__ mu_dev,
                                                  double* __restrict__ part_lam) {
  __shared__ double red[8];
  const int64_t N = (int64_t)c.h * c.w * c.b;
  const double mud = *mu_dev;
  const float mu = (float)mud, imu = (float)(1.0 / mud);
  const bool has_ga = c.gaZ != nullptr;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N; q += (int64_t)gridDim.x * blockDim.x) {
    const float aG1 = has_ga ? c.gaG1[q] : 0.f, aG2 = has_ga ? c.gaG2[q] : 0.f;
    const float aS = has_ga ? c.gaS[q] : 0.f, aZ = has_ga ? c.gaZ[q] : 0.f;
    // Gamma1' = Gamma1 + mu (O - L - S'), Gamma2' = Gamma2 + mu (L - Z')
    float gL = (c.gX ? c.gX[q] : 0.f) + mu * aG2 - mu * aG1;
    float gO = mu * aG1;
    const float gS = aS - mu * aG1;
    // S' = R_{lambda/mu}(O - L + Gamma1/mu)
    const float s1 = c.S1[q];
    const float gV = (s1 != 0.f) ? gS : 0.f;
    acc -= (s1 > 0.f) ? (double)gV : (s1 < 0.f) ? -(double)gV : 0.0;
    gO += gV;
    gL -= gV;
    c.gbG1[q] = aG1 + gV * imu;
    c.gbG2[q] = aG2;
    c.gL[q] = gL;
    c.gZp[q] = aZ - mu * aG2;
    c.gY[q] += gO;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t o3 = n * c.ts + q, oa = n * c.as + q;
      const float aF = has_ga ? c.gaF[o3] : 0.f, aE = has_ga ? c.gaE[o3] : 0.f;
      const float aG3 = has_ga ? c.gaG3[o3] : 0.f, aG4 = has_ga ? c.gaG4[o3] : 0.f;
      // Gamma3' = Gamma3 + mu (G - F'), Gamma4' = Gamma4 + mu (E' - F')
      c.gFp[o3] = aF - mu * aG3 - mu * aG4;
      c.dirE[oa] = aE + mu * aG4;
      c.A[oa] = c.F1[o3] - c.G4[o3] * imu;
      c.gbG3[o3] = aG3;
      c.gbG4[o3] = aG4;
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part_lam[blockIdx.x] = acc * (1.0 / mud);
}

// gA_n (the t-SVT cotangent, component stride as) is added to gF'; then
// F' = R_{tau/mu}(U): gU = 1[F' != 0] gF';  U = (G + Gamma3/mu + E + Gamma4/mu)/2
// gG_n = mu ga.Gamma3_n + gU_n / 2 is written over gF'.
__global__ void __launch_bounds__(256) k_vjp_shrinkf(VjpCube c, const float* __restrict__ gA,
                                                     const double* __restrict__ mu_dev,
                                                     double* __restrict__ part_tau) {
  __shared__ double red[8];
  const int64_t N = (int64_t)c.h * c.w * c.b;
  const double mud = *mu_dev;
  const float mu = (float)mud, imu = (float)(1.0 / mud);
  const bool has_ga = c.gaZ != nullptr;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N; q += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t o3 = n * c.ts + q;
      const float ga = gA[n * c.as + q];
      const float gF = c.gFp[o3] + ga;
      const float f1 = c.F1[o3];
      const float gU = (f1 != 0.f) ? gF : 0.f;
      acc -= (f1 > 0.f) ? (double)gU : (f1 < 0.f) ? -(double)gU : 0.0;
      const float hU = 0.5f * gU;
      c.gbG4[o3] += (hU - ga) * imu;
      c.gbG3[o3] += hU * imu;
      c.gbE[o3] = hU;
      c.gFp[o3] = (has_ga ? mu * c.gaG3[o3] : 0.f) + hU;
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part_tau[blockIdx.x] = acc * (1.0 / mud);
}

// T = gZ' + sum_n w_n D_n^T gG_n,  (D_n^T y)[v] = y[v - e_n] - y[v]
__global__ void __launch_bounds__(256) k_vjp_divt(VjpCube c, float* __restrict__ T, float w1, float w2, float w3) {
  const int h = c.h, w = c.w, b = c.b;
  const int64_t hw = (int64_t)h * w, N = hw * b;
  const float* G0 = c.gFp;
  const float* G1 = c.gFp + c.ts;
  const float* G2 = c.gFp + 2 * c.ts;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N; q += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(q % w);
    const int i = (int)((q / w) % h);
    const int j = (int)(q / hw);
    const int64_t qh = (i == 0) ? q + (int64_t)(h - 1) * w : q - w;
    const int64_t qw = (x == 0) ? q + (w - 1) : q - 1;
    const int64_t qb = (j == 0) ? q + (int64_t)(b - 1) * hw : q - hw;
    T[q] = c.gZp[q] + w1 * (G0[qh] - G0[q]) + w2 * (G1[qw] - G1[q]) + w3 * (G2[qb] - G2[q]);
  }
}

// With gT the solved cotangent of T_z = mu L + mu D_w^* F + Gamma2 - D_w^* Gamma3:
//   gL += mu gT;  gb.F_n = mu w_n D_n gT;  gb.Gamma2 += gT;  gb.Gamma3_n -= w_n D_n gT
// and of L = (O - S + Z + (Gamma1 - Gamma2)/mu)/2:
//   gY += gL/2;  gb.S = -gL/2;  gb.Z = gL/2;  gb.Gamma1 += gL/(2mu);  gb.Gamma2 -= gL/(2mu)
// (from the initial state, Z = O: gY also receives gb.Z, so gY += gL).
__global__ void __launch_bounds__(256) k_vjp_pre(VjpCube c, const float* __restrict__ gT, float w1, float w2,
                                                 float w3, const double* __restrict__ mu_dev) {
  const int h = c.h, w = c.w, b = c.b;
  const int64_t hw = (int64_t)h * w, N = hw * b;
  const double mud = *mu_dev;
  const float mu = (float)mud, imu = (float)(1.0 / mud);
  const float wn[3] = {w1, w2, w3};
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N; q += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(q % w);
    const int i = (int)((q / w) % h);
    const int j = (int)(q / hw);
    const int64_t qn[3] = {(i == h - 1) ? q - (int64_t)(h - 1) * w : q + w, (x == w - 1) ? q - (w - 1) : q + 1,
                           (j == b - 1) ? q - (int64_t)(b - 1) * hw : q + hw};
    const float t = gT[q];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t o3 = n * c.ts + q;
      const float dt = wn[n] * (gT[qn[n]] - t);
      c.gbF[o3] = mu * dt;
      c.gbG3[o3] -= dt;
    }
    const float gL = c.gL[q] + mu * t;
    const float hL = 0.5f * gL;
    c.gY[q] += c.initial ? gL : hL;
    c.gbS[q] = -hL;
    c.gbZ[q] = hL;
    c.gbG1[q] += hL * imu;
    c.gbG2[q] += t - hL * imu;
  }
}

// One block per cube: gw[c] += (tau, alpha, lambda) cotangents, summed in a
// fixed order from the block partials and the per-column threshold terms.
__global__ void k_vjp_finish(const double* __restrict__ part, const double* __restrict__ acon,
                             const int64_t* __restrict__ acon_range, int n_cubes, double* __restrict__ gw) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  if (c >= n_cubes) return;
  const double* p = part + (int64_t)c * 2 * LRSTV_PARTS;
  double st = 0.0, sl = 0.0, sa = 0.0;
  for (int k = threadIdx.x; k < LRSTV_PARTS; k += blockDim.x) {
    st += p[k];
    sl += p[LRSTV_PARTS + k];
  }
  const int64_t a0 = acon_range[2 * c], a1 = acon_range[2 * c + 1];
  for (int64_t k = a0 + threadIdx.x; k < a1; k += blockDim.x) sa += acon[k];
  st = block_sum(st, red);
  sl = block_sum(sl, red);
  sa = block_sum(sa, red);
  if (threadIdx.x == 0) {
    gw[3 * c + 0] += st;
    gw[3 * c + 1] += sa;
    gw[3 * c + 2] += sl;
  }
}

__global__ void k_sum_ranges(const double* __restrict__ acon, const int64_t* __restrict__ range, int n,
                             double* __restrict__ out) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  if (c >= n) return;
  double a = 0.0;
  for (int64_t k = range[2 * c] + threadIdx.x; k < range[2 * c + 1]; k += blockDim.x) a += acon[k];
  a = block_sum(a, red);
  if (threadIdx.x == 0) out[c] = a;
}

// ------------------------------------------------------------ launchers ---
static int grid_for(int64_t N) {
  int g = (int)((N + 255) / 256);
  return g > 8192 ? 8192 : (g < 1 ? 1 : g);
}

void launch_vjp_post(const VjpCube& c, const double* mu, double* part_lam, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_post, dim3(LRSTV_PARTS), dim3(256), 0, s, c, mu, part_lam);
}

void launch_vjp_shrinkf(const VjpCube& c, const float* gA, const double* mu, double* part_tau, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_shrinkf, dim3(LRSTV_PARTS), dim3(256), 0, s, c, gA, mu, part_tau);
}

void launch_vjp_divt(const VjpCube& c, float* T, const double w[3], hipStream_t s) {
  const int64_t N = (int64_t)c.h * c.w * c.b;
  hipLaunchKernelGGL(k_vjp_divt, dim3(grid_for(N)), dim3(256), 0, s, c, T, (float)w[0], (float)w[1], (float)w[2]);
}

void launch_vjp_pre(const VjpCube& c, const float* gT, const double w[3], const double* mu, hipStream_t s) {
  const int64_t N = (int64_t)c.h * c.w * c.b;
  hipLaunchKernelGGL(k_vjp_pre, dim3(grid_for(N)), dim3(256), 0, s, c, gT, (float)w[0], (float)w[1], (float)w[2],
                     mu);
}

void launch_vjp_finish(const double* part, const double* acon, const int64_t* acon_range, int n_cubes, double* gw,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_finish, dim3(n_cubes), dim3(256), 0, s, part, acon, acon_range, n_cubes, gw);
}

void launch_sum_ranges(const double* acon, const int64_t* range, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_ranges, dim3(n), dim3(256), 0, s, acon, range, n, out);
}

}  // namespace lrstv
