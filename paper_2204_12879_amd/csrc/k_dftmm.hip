// Transforms of the Z-update (Sec. III-C, the FFT diagonalisation of the
// X-subproblem) along w and h as products with the DFT matrix on the matrix
// cores, for lengths with a large prime factor (dft_mm_len).  The Stockham
// FFT's direct-DFT stage of a prime p reads O(p) LDS values per element; the
// product issues 6n (complex, 3M form) or 2n (real, even / odd halves)
// matrix-core flops per element of a length-n transform, at the FP32 matrix
// rate.  The results are the same DFTs (up to rounding) as the FFT path's.
//
// A strip is 16 rows (w, one wave per block) or 16 columns (h, four waves
// per block sharing it), staged in LDS.  The DFT-matrix operand comes from an LDS table of
// (cos, sin)(2 pi m / n); the index k j mod n of a lane is advanced by
// 4 k mod n per step of four along the contraction.  v_mfma_f32_16x16x4f32:
// lane l holds A(l % 16, l / 16), B(l / 16, l % 16) and the accumulator
// elements C(4 (l / 16) + e, l % 16), e = 0..3.
//
// This file is compiled with the matrix-core accumulators in VGPRs
// (-mllvm -amdgpu-mfma-vgpr-form): with them in AGPRs the register
// allocator copied accumulators between AGPRs on every step of these loops,
// whose operand index is a loop-carried value.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace lrstv {

LRSTV_DEV f32x4 mfma16(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// (cos, sg sin)(2 pi m / n) for m < n, from FP64 values rounded once
LRSTV_DEV void mm_table(float2* tab, int n, double sg) {
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double sv, cv;
    sincospi(2.0 * (double)m / (double)n, &sv, &cv);
    tab[m] = make_float2((float)cv, (float)(sg * sv));
  }
}
// smallest row stride >= n that is 2 mod 32: the operand reads of 16 rows x
// two columns by each half-wave fall on distinct banks
__host__ __device__ inline int mm_ld(int n) { return n + (((2 - n) % 32) + 32) % 32; }

// ------------------------------------------------------------ along h ---
// Complex transform of spec [b][h][wc] along h (sign -1 forward, +1 inverse,
// unnormalised), in place: X(k, g) = sum_i F(k, i) S(i, g) over the flat
// columns g = j wc + c, F(k, i) = exp(sign 2 pi i k i / h), in the 3M form
// P1 = Re F Re S, P2 = Im F Im S, P3 = (Re F + Im F)(Re S + Im S),
// Re X = P1 - P2, Im X = P3 - P1 - P2.  A strip is 16 columns and all h rows,
// read whole into LDS before any of its outputs is written.

// The wave's NP row tiles m = wv, wv + 4, .. of the strip in LDS, outputs to
// base (column cl).  The operands of the next step are read before the
// products of the current one.
template <int NP>
LRSTV_DEV void dftmm_h_tiles(const float2* tab, const float* pr, const float* pim, float2* base, bool ok, int wv,
                             int h, int h4, int wc, int cl, int rq) {
  f32x4 p1[NP], p2[NP], p3[NP];
  int idx[NP], stp[NP];
  float2 f[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int k = 16 * (wv + 4 * m) + cl;   // the lane's row of F, its column rq at the first step
    p1[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    p2[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    p3[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    idx[m] = (k * rq) % h;
    stp[m] = (4 * k) % h;
    f[m] = tab[idx[m]];
  }
  float br = pr[16 * rq + cl], bi = pim[16 * rq + cl];
#pragma unroll 1
  for (int i0 = 0; i0 < h4; i0 += 4) {
    const int i1 = i0 + 4 < h4 ? i0 + 4 : i0;   // the next step (the last step reads its own again)
    const float brn = pr[16 * (i1 + rq) + cl], bin = pim[16 * (i1 + rq) + cl];
    float2 fn[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      idx[m] += stp[m];
      if (idx[m] >= h) idx[m] -= h;
      fn[m] = tab[idx[m]];
    }
    const float bs = br + bi;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      p1[m] = mfma16(f[m].x, br, p1[m]);
      p2[m] = mfma16(f[m].y, bi, p2[m]);
      p3[m] = mfma16(f[m].x + f[m].y, bs, p3[m]);
    }
    br = brn;
    bi = bin;
#pragma unroll
    for (int m = 0; m < NP; ++m) f[m] = fn[m];
  }
  if (!ok) return;
#pragma unroll
  for (int m = 0; m < NP; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 16 * (wv + 4 * m) + 4 * rq + e;
      if (k < h) base[(int64_t)k * wc] = make_float2(p1[m][e] - p2[m][e], p3[m][e] - p1[m][e] - p2[m][e]);
    }
}

// Block of four waves per strip: the 256 threads stage it, wave wv forms row
// tiles wv, wv + 4, wv + 8 (ceil(h / 16) <= 12).
LRSTV_DEV void dftmm_h_body(int bid, int nblk, float* sm, float2* __restrict__ spec, int h, int wc, int b, int sign) {
  const int h4 = (h + 3) & ~3;
  float2* tab = reinterpret_cast<float2*>(sm);
  float* pr = sm + 2 * h;   // planes [h4][16]
  float* pim = pr + 16 * h4;
  mm_table(tab, h, (double)sign);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, cl = lane & 15, rq = lane >> 4;
  const int nrt = (h + 15) >> 4, ntw = wv < nrt ? (nrt - wv + 3) >> 2 : 0;
  const int64_t ncol = (int64_t)b * wc, plane = (int64_t)h * wc;
  const int64_t nstrip = (ncol + 15) >> 4;
  for (int64_t st = xcd_block(bid, nblk); st < nstrip; st += nblk) {
    const int64_t g = st * 16 + cl;
    const bool ok = g < ncol;
    const int64_t j = ok ? g / wc : 0;
    float2* base = spec + j * plane + (ok ? g - j * wc : 0);
    __syncthreads();   // the table is written; the last strip's plane reads are done
    for (int i = t >> 4; i < h4; i += 16) {
      const float2 v = (ok && i < h) ? base[(int64_t)i * wc] : make_float2(0.f, 0.f);
      pr[16 * i + cl] = v.x;
      pim[16 * i + cl] = v.y;
    }
    __syncthreads();
    switch (ntw) {
      case 1: dftmm_h_tiles<1>(tab, pr, pim, base, ok, wv, h, h4, wc, cl, rq); break;
      case 2: dftmm_h_tiles<2>(tab, pr, pim, base, ok, wv, h, h4, wc, cl, rq); break;
      case 3: dftmm_h_tiles<3>(tab, pr, pim, base, ok, wv, h, h4, wc, cl, rq); break;
      default: break;
    }
  }
}

// ------------------------------------------------------------ along w ---
// Real forward transform of the rows of T (nrows rows of length w) into the
// half spectrum (s = w/2 + 1 values per row) with the even / odd parts
// P_x = T_x + T_{w-x}, Q_x = T_x - T_{w-x} (P_0 = T_0, and P_{w/2} = T_{w/2}
// for even w):  Re Y_k = sum_{x<s} P_x cos(2 pi x k / w),
// Im Y_k = -sum_{x<s} Q_x sin(2 pi x k / w).  A strip is 16 consecutive
// rows, one contiguous range of T.  NCT = ceil(s / 16) column tiles.
template <int NCT>
LRSTV_DEV void dftmm_rw_tiles(int bid, int nblk, float* sm, const float* __restrict__ T, float2* __restrict__ spec,
                              int nrows, int w) {
  const int s = w / 2 + 1, s4 = (s + 3) & ~3, ld = mm_ld(w);
  float2* tab = reinterpret_cast<float2*>(sm);
  float* ts = sm + 2 * w;   // [16][ld]
  mm_table(tab, w, 1.0);
  const int lane = threadIdx.x, cl = lane & 15, rq = lane >> 4;
  const int nstrip = (nrows + 15) >> 4;
  int stp[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) stp[c] = (4 * (16 * c + cl)) % w;
  for (int st = bid; st < nstrip; st += nblk) {
    const int r0 = 16 * st, nr = nrows - r0 < 16 ? nrows - r0 : 16;
    const float* src = T + (int64_t)r0 * w;
    __syncthreads();
    {
      int row = lane / w, col = lane - (lane / w) * w;   // element e = row w + col of the strip
      for (int e = lane; e < nr * w; e += 64) {
        ts[row * ld + col] = src[e];
        col += 64;
        while (col >= w) {
          col -= w;
          ++row;
        }
      }
    }
    __syncthreads();
    f32x4 are[NCT], aim[NCT];
    int idx[NCT];
    float2 t[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      are[c] = f32x4{0.f, 0.f, 0.f, 0.f};
      aim[c] = f32x4{0.f, 0.f, 0.f, 0.f};
      idx[c] = ((16 * c + cl) * rq) % w;   // x = rq, k = 16 c + cl
      t[c] = tab[idx[c]];
    }
    // P_x, Q_x of the lane's row cl at x (the next step's read before the
    // current step's products)
    auto pq = [&](int x, float& P, float& Q) {   // x < s4 <= w - 1 (w >= 8)
      const float a = ts[cl * ld + x];
      const float mv = (x > 0 && 2 * x != w) ? ts[cl * ld + (w - x)] : 0.f;
      P = x < s ? a + mv : 0.f;
      Q = x < s ? a - mv : 0.f;
    };
    float P, Q;
    pq(rq, P, Q);
#pragma unroll 1
    for (int x0 = 0; x0 < s4; x0 += 4) {
      float Pn, Qn;
      pq((x0 + 4 < s4 ? x0 + 4 : x0) + rq, Pn, Qn);
      float2 tn[NCT];
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        idx[c] += stp[c];
        if (idx[c] >= w) idx[c] -= w;
        tn[c] = tab[idx[c]];
      }
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        are[c] = mfma16(P, t[c].x, are[c]);
        aim[c] = mfma16(Q, t[c].y, aim[c]);
      }
      P = Pn;
      Q = Qn;
#pragma unroll
      for (int c = 0; c < NCT; ++c) t[c] = tn[c];
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * rq + e, k = 16 * c + cl;
        if (r < nr && k < s) spec[(int64_t)(r0 + r) * s + k] = make_float2(are[c][e], -aim[c][e]);
      }
  }
}

// Inverse of dftmm_rw_tiles times `scale`, into the real rows of Z, with the
// Hermitian completion of the half spectrum (c_k = 1 for k = 0 and k = w/2,
// else 2):  C_x = sum_{k<s} c_k Re X_k cos(2 pi k x / w),
// S_x = sum_{k<s} c_k Im X_k sin(2 pi k x / w), z_x = C_x - S_x and
// z_{w-x} = C_x + S_x for x < s.  With `part`, also the FP64 sum of
// (Z_new - Z_old)^2 over the block (slot R_DUAL_Z of the block).
template <int NCT>
LRSTV_DEV void dftmm_irw_tiles(int bid, int nblk, float* sm, const float2* __restrict__ spec, float* __restrict__ Z,
                               int nrows, int w, float scale, double* __restrict__ part) {
  const int s = w / 2 + 1, s4 = (s + 3) & ~3, ld = mm_ld(s4);
  float2* tab = reinterpret_cast<float2*>(sm);
  float* xr = sm + 2 * w;   // planes [16][ld]
  float* xi = xr + 16 * ld;
  mm_table(tab, w, 1.0);
  const int lane = threadIdx.x, cl = lane & 15, rq = lane >> 4;
  const int nstrip = (nrows + 15) >> 4;
  int stp[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) stp[c] = (4 * (16 * c + cl)) % w;
  double acc = 0.0;
  for (int st = bid; st < nstrip; st += nblk) {
    const int r0 = 16 * st, nr = nrows - r0 < 16 ? nrows - r0 : 16;
    const float2* src = spec + (int64_t)r0 * s;
    __syncthreads();
    {
      int row = lane / s, col = lane - (lane / s) * s;
      for (int e = lane; e < nr * s; e += 64) {
        const float2 v = src[e];
        const float ck = (col == 0 || 2 * col == w) ? 1.f : 2.f;
        xr[row * ld + col] = ck * v.x;
        xi[row * ld + col] = ck * v.y;
        col += 64;
        while (col >= s) {
          col -= s;
          ++row;
        }
      }
    }
    __syncthreads();
    f32x4 cc[NCT], ss[NCT];
    int idx[NCT];
    float2 t[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      cc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
      ss[c] = f32x4{0.f, 0.f, 0.f, 0.f};
      idx[c] = ((16 * c + cl) * rq) % w;   // k = rq, x = 16 c + cl
      t[c] = tab[idx[c]];
    }
    float ar = xr[cl * ld + rq], ai = xi[cl * ld + rq];
#pragma unroll 1
    for (int k0 = 0; k0 < s4; k0 += 4) {
      const int kn = (k0 + 4 < s4 ? k0 + 4 : k0) + rq;   // the next step's column
      const float arn = xr[cl * ld + kn], ain = xi[cl * ld + kn];
      float2 tn[NCT];
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        idx[c] += stp[c];
        if (idx[c] >= w) idx[c] -= w;
        tn[c] = tab[idx[c]];
      }
      const bool kin = k0 + rq < s;   // columns s .. s4 - 1 of the planes are not staged
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        cc[c] = mfma16(kin ? ar : 0.f, t[c].x, cc[c]);
        ss[c] = mfma16(kin ? ai : 0.f, t[c].y, ss[c]);
      }
      ar = arn;
      ai = ain;
#pragma unroll
      for (int c = 0; c < NCT; ++c) t[c] = tn[c];
    }
    // the strip's rows of Z through LDS (the planes are free now): old values
    // in, new values out, both as one contiguous range
    float* zb = xr;   // [16][w] in 32 ld >= 16 w + 32 floats
    float* zg = Z + (int64_t)r0 * w;
    __syncthreads();
    if (part)
      for (int e = lane; e < nr * w; e += 64) zb[e] = zg[e];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * rq + e, x = 16 * c + cl;
        if (r < nr && x < s) {
          float* zr = zb + r * w;
          const float z0 = scale * (cc[c][e] - ss[c][e]);
          if (part) {
            const double d = (double)z0 - (double)zr[x];
            acc += d * d;
          }
          zr[x] = z0;
          if (x > 0 && 2 * x != w) {
            const float z1 = scale * (cc[c][e] + ss[c][e]);
            if (part) {
              const double d = (double)z1 - (double)zr[w - x];
              acc += d * d;
            }
            zr[w - x] = z1;
          }
        }
      }
    __syncthreads();
    for (int e = lane; e < nr * w; e += 64) zg[e] = zb[e];
  }
  if (part) {
    acc = warp_sum(acc);
    if (lane == 0) part[R_DUAL_Z * LRSTV_PARTS + bid] = acc;
  }
}

// the instantiations for the length's column-tile count ceil((w/2 + 1) / 16) (1 .. 9)
#define LRSTV_MMW_CASES(F) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9)
LRSTV_DEV void dftmm_rw_body(int bid, int nblk, float* sm, const float* __restrict__ T, float2* __restrict__ spec,
                             int nrows, int w) {
  switch ((w / 2 + 16) >> 4) {
#define LRSTV_MMW(N) \
  case N: dftmm_rw_tiles<N>(bid, nblk, sm, T, spec, nrows, w); break;
    LRSTV_MMW_CASES(LRSTV_MMW)
#undef LRSTV_MMW
    default: break;
  }
}
LRSTV_DEV void dftmm_irw_body(int bid, int nblk, float* sm, const float2* __restrict__ spec, float* __restrict__ Z,
                              int nrows, int w, float scale, double* __restrict__ part) {
  switch ((w / 2 + 16) >> 4) {
#define LRSTV_MMW(N) \
  case N: dftmm_irw_tiles<N>(bid, nblk, sm, spec, Z, nrows, w, scale, part); break;
    LRSTV_MMW_CASES(LRSTV_MMW)
#undef LRSTV_MMW
    default: break;
  }
}
#undef LRSTV_MMW_CASES

// ------------------------------------------------------------- kernels ---
__global__ void __launch_bounds__(256) k_dftmm_h(float2* __restrict__ spec, int h, int wc, int b, int sign) {
  extern __shared__ float smf[];
  dftmm_h_body(blockIdx.x, gridDim.x, smf, spec, h, wc, b, sign);
}
__global__ void __launch_bounds__(64) k_dftmm_rw(const float* __restrict__ T, float2* __restrict__ spec, int nrows,
                                                 int w) {
  extern __shared__ float smf[];
  dftmm_rw_body(blockIdx.x, gridDim.x, smf, T, spec, nrows, w);
}
__global__ void __launch_bounds__(64) k_dftmm_irw(const float2* __restrict__ spec, float* __restrict__ Z, int nrows,
                                                  int w, float scale, double* __restrict__ part) {
  extern __shared__ float smf[];
  dftmm_irw_body(blockIdx.x, gridDim.x, smf, spec, Z, nrows, w, scale, part);
}

// Batched: the cubes whose CubeGeo::mm bit is set, each over its own block
// range (the grid it would get alone, so a cube's results do not depend on
// the other cubes).
__global__ void __launch_bounds__(256) k_dftmm_h_batch(BatchTab bt, float2* __restrict__ spec, int sign) {
  extern __shared__ float smf[];
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (!(g.mm & 1)) return;
  dftmm_h_body(q.bid, q.nblk, smf, spec + g.spec_off, g.h, g.w / 2 + 1, g.b, sign);
}
__global__ void __launch_bounds__(64) k_dftmm_rw_batch(BatchTab bt, const float* __restrict__ T,
                                                       float2* __restrict__ spec) {
  extern __shared__ float smf[];
  const CubeSel q = select_cube(bt);
  if (cube_halted(bt, q.c)) return;
  const CubeGeo g = uniform_geo(bt.geo, q.c);
  if (!(g.mm & 2)) return;
  dftmm_rw_body(q.bid, q.nblk, smf, T + g.off, spec + g.spec_off, g.h * g.b, g.w);
}
__global__ void __launch_bounds__(64) k_dftmm_irw_batch(BatchTab bt, const float2* __restrict__ spec,
                                                        float* __restrict__ Z, double* __restrict__ part) {
  extern __shared__ float smf[];
  const int c = blockIdx.x / LRSTV_PARTS;
  if (cube_halted(bt, c)) return;
  const CubeGeo g = uniform_geo(bt.geo, c);
  if (!(g.mm & 2)) return;
  dftmm_irw_body(blockIdx.x - c * LRSTV_PARTS, LRSTV_PARTS, smf, spec + g.spec_off, Z + g.off, g.h * g.b, g.w,
                 1.0f / ((float)g.h * (float)g.w), part ? part + (int64_t)c * R_COUNT * LRSTV_PARTS : nullptr);
}

// ----------------------------------------------------------- launchers ---
size_t dftmm_lds_h(int h) { return ((size_t)2 * h + (size_t)32 * ((h + 3) & ~3)) * sizeof(float); }
size_t dftmm_lds_w(int w) { return ((size_t)2 * w + (size_t)16 * mm_ld(w)) * sizeof(float); }
size_t dftmm_lds_wi(int w) { return ((size_t)2 * w + (size_t)32 * mm_ld(((w / 2 + 1) + 3) & ~3)) * sizeof(float); }
int dftmm_blocks_h(int h, int w, int b) {
  const int64_t g = ((int64_t)b * (w / 2 + 1) + 15) / 16;
  return (int)(g < 8192 ? g : 8192);
}
int dftmm_blocks_w(int h, int w, int b) {
  const int64_t g = ((int64_t)h * b + 15) / 16;
  return (int)(g < 8192 ? g : 8192);
}

void launch_dftmm_h(float2* spec, int h, int w, int b, int sign, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_h, dim3(dftmm_blocks_h(h, w, b)), dim3(256), dftmm_lds_h(h), s, spec, h, w / 2 + 1, b,
                     sign);
}
void launch_dftmm_rw(const float* T, float2* spec, int h, int w, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_rw, dim3(dftmm_blocks_w(h, w, b)), dim3(64), dftmm_lds_w(w), s, T, spec, h * b, w);
}
// LRSTV_PARTS blocks, as the batched form gives every cube (the residual
// partials of a cube are the same alone and in a batch)
void launch_dftmm_irw(const float2* spec, float* Z, int h, int w, int b, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_irw, dim3(LRSTV_PARTS), dim3(64), dftmm_lds_wi(w), s, spec, Z, h * b, w,
                     1.0f / ((float)h * (float)w), part);
}
void launch_dftmm_h_batch(const BatchTab& bt, float2* spec, int sign, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_h_batch, dim3(bt.nblocks), dim3(256), bt.lds_mm_h, s, bt, spec, sign);
}
void launch_dftmm_rw_batch(const BatchTab& bt, const float* T, float2* spec, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_rw_batch, dim3(bt.nblocks), dim3(64), bt.lds_mm_w, s, bt, T, spec);
}
void launch_dftmm_irw_batch(const BatchTab& bt, const float2* spec, float* Z, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_dftmm_irw_batch, dim3(bt.nc * LRSTV_PARTS), dim3(64), bt.lds_mm_wi, s, bt, spec, Z, part);
}

}  // namespace lrstv
