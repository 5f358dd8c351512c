// Shared device helpers and descriptor structs of the LRSTV HIP library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LRSTV_DEV __device__ __forceinline__

// Largest cube side (LRSTV_MAX_SIDE of the public header; checked there).
#define LRSTV_MAX_SIDE_DEV 512

namespace lrstv {

// ---------------------------------------------------------------- complex ---
LRSTV_DEV float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
LRSTV_DEV float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
LRSTV_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
LRSTV_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
LRSTV_DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
LRSTV_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

LRSTV_DEV float soft_threshold(float x, float t) {
  // R_t(x) = sign(x) max(|x| - t, 0)
  float m = fabsf(x) - t;
  return m > 0.f ? copysignf(m, x) : 0.f;
}

// Cube owning block `blk` of a batched launch: bstart[c] <= blk < bstart[c+1].
LRSTV_DEV int find_cube(const int* __restrict__ bstart, int nc, int blk) {
  int lo = 0, hi = nc;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (bstart[mid] <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------- reductions ---
LRSTV_DEV double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
LRSTV_DEV double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
LRSTV_DEV float warp_sumf(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave-wide float sum with DPP row operations (quad permutes, row mirrors,
// row broadcasts); the total is read from lane 63 and returned to all lanes.
// The DPP builtin moves 32-bit integers, hence the bit casts.
template <int CTRL, int ROWMASK>
LRSTV_DEV float dpp_moved(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, false));
}
LRSTV_DEV float wave_sumf_dpp(float v) {
  v += dpp_moved<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_moved<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_moved<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_moved<0x140, 0xf>(v);   // row_mirror
  v += dpp_moved<0x142, 0xa>(v);   // row_bcast:15 -> rows 1, 3
  v += dpp_moved<0x143, 0xc>(v);   // row_bcast:31 -> rows 2, 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Double-precision wave sum by the same DPP pattern, both 32-bit halves
// moved with the same control.
template <int CTRL, int ROWMASK>
LRSTV_DEV double dpp_moved_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
LRSTV_DEV double wave_sum_dpp(double v) {
  v += dpp_moved_d<0xb1, 0xf>(v);
  v += dpp_moved_d<0x4e, 0xf>(v);
  v += dpp_moved_d<0x141, 0xf>(v);
  v += dpp_moved_d<0x140, 0xf>(v);
  v += dpp_moved_d<0x142, 0xa>(v);
  v += dpp_moved_d<0x143, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Values known to be equal in every lane, moved to scalar registers.
LRSTV_DEV float uniform_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
LRSTV_DEV double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// An opaque copy: the compiler may not assume it equals v, so values derived
// from it inside a loop are recomputed there instead of being kept live
// across the loop.
LRSTV_DEV int opaque_i(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Block barrier for LDS traffic only: waits for this wave's LDS (and
// scalar) operations, not for its global stores, which nothing in the block
// reads back.  Every wave of the block must reach it.
LRSTV_DEV void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Block-wide sum in a fixed order (deterministic).  `scratch` holds
// blockDim/64 doubles.  Every thread gets the result.
LRSTV_DEV double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = warp_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += scratch[i];
  return r;
}
LRSTV_DEV double block_max(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = warp_max(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r = fmax(r, scratch[i]);
  return r;
}

// ------------------------------------------------------------ descriptors ---
// Residual slots per cube (same order as the public LRSTV_NRES list).
enum { R_INF_OLS = 0, R_INF_LZ, R_FRO_OLS, R_FRO_LZ, R_FRO_DZF, R_FRO_EF, R_DUAL_Z, R_COUNT };

// Number of per-block partials each residual-producing kernel writes.
#define LRSTV_PARTS 512

// One Fourier slice of one gradient tensor of one cube (or of one tensor of
// the standalone t-SVT batch).
struct SliceDesc {
  int h, w;          // slice is h x w complex, row-major, planar (re plane, im plane)
  int n1, m1;        // min / max of (h, w)
  int tall;          // 1 if h >= w (Gram = M^H M), else Gram = M M^H
  int cube;          // owning cube
  float fw;          // Fourier weight of the slice: (1 or 2) / b, 2 when the slice
                     // stands for itself and its conjugate partner k' = b - k
  int64_t a_off;     // float offset of the re plane; im plane at a_off + h*w
  int64_t g_off;     // float2 offset of the packed lower Gram / reflector scratch
  int64_t v_off;     // float offset of V (planar, n1 x n1, re then im)
  int64_t b_off;     // float offset of the back-projection intermediate (planar)
  int64_t t_off;     // double offset of the tridiagonal scratch (d, |e|, phase re/im)
  int64_t x_off;     // double offset of the eigenvector scratch (3 n1 x n1)
  int64_t f_off;     // float offset of the n1 shrink factors
  int64_t y_off;     // float offset of the block-reflector T factors
                     // (ceil((n1-1)/64) blocks of 64 x 64 complex, planar)
  int keep;          // > 0: keep the `keep` largest eigenpairs of the matrix
                     // (Tucker projectors) instead of those above the threshold
  int prio;          // 1: a slice of the group that runs after the first round of
                     // compute units; its eigen-solve and back-transform waves
                     // issue at raised priority
};

}  // namespace lrstv
