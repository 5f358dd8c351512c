// Host-side launcher declarations shared by the kernel files and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "timer.hpp"

namespace lrstv {

struct Weights {
  double tau, alpha, lam;
  double w[3];
  int iso;   // 1: isotropic gradient term (group soft-threshold per voxel)
  double beta;   // > 0: explicit noise term beta ||N||^2 (N read and updated)
};


struct SliceDesc;

// ---- packed ragged batches: one launch per phase --------------------------
struct CubeGeo {
  int h, w, b;
  int nb_w, cw_h;          // rows per block of the w FFT, columns per block of the h FFT
  int nb_wi;               // rows per block of the inverse w FFT
  int mm;                  // bit 0: the h transforms, bit 1: the w transforms run as
                           // DFT-matrix products (dft_mm_len)
  int64_t off;             // element offset of the cube in the packed batch
  int64_t spec_off;        // complex offset of its half spectrum
  int64_t slice_base;      // float offset of its Fourier slices
};
enum Phase { PH_LRHS = 0, PH_RFFT_W, PH_FFT_H, PH_TRI_B, PH_BAND_DFT, PH_PARTS, PH_COUNT };
// Block ranges of one phase: cube c owns blocks [bstart[c], bstart[c+1]).
struct BatchTab {
  const CubeGeo* geo;      // device [nc]
  const int* bstart;       // device [nc + 1]
  int nc, nblocks;
  size_t lds_w, lds_h;     // dynamic LDS of the w / h FFT phases (max over cubes)
  size_t lds_wi;           // and of the inverse w FFT
  int max_b;               // largest band count over cubes
  int reg_h_mask;          // h FFT lengths present that run in registers (bit 0: 64, 1: 128, 2: 256)
  int stockham_h;          // 1 when some cube's h FFT runs through the LDS Stockham path
  int reg_w_mask, stockham_w;   // the same for the w transforms
  int mm_h, mm_w;          // 1 when some cube's h (w) transforms are DFT-matrix products
  size_t lds_mm_h, lds_mm_w, lds_mm_wi;   // their dynamic LDS (max over those cubes)
  const int* halt;         // device [nc] or NULL: a cube whose entry is non-zero
                           // has met the stopping test; every phase skips it
};
// Block-uniform early exit of a batched phase for a halted cube.
__device__ __forceinline__ bool cube_halted(const BatchTab& bt, int c) { return bt.halt && bt.halt[c] != 0; }
// Bit of an FFT length that runs in registers (64, 128, 256), else 0.
__host__ __device__ inline int fft_h_reg_bit(int h) { return h == 64 ? 1 : h == 128 ? 2 : h == 256 ? 4 : 0; }
// Lengths whose transform along h (up to 192) or w (up to 256) runs as a
// product with the DFT matrix on the matrix cores instead of the Stockham
// FFT: those with a prime factor p >= 17, or p = 11, 13 and n <= 144 (the
// Stockham direct-DFT stage costs O(p) LDS reads per element; the product
// O(n) matrix-core flops).  Measured per length (Z-solve of 100 bands): the
// product is faster for 77, 78, 88, 91, 110, 121, 143 and every p >= 17,
// the FFT for smooth lengths from 80 up and for 156.
constexpr int kMmMaxH = 192, kMmMaxW = 256, kMmMinPrime = 17, kMmMidPrime = 11, kMmMidMax = 144;
inline bool dft_mm_len(int n, int nmax) {
  if (n > nmax || fft_h_reg_bit(n) != 0) return false;
  int p = 1, m = n;
  for (int d = 2; d * d <= m; ++d)
    while (m % d == 0) {
      p = d;
      m /= d;
    }
  if (m > 1) p = m;
  return p >= kMmMinPrime || (p >= kMmMidPrime && n <= kMmMidMax);
}
// Base pointers of the packed batch (gradient-shaped arrays and A: 3
// components spaced by ts).
struct BatchPtrs {
  const float* O;
  float *L, *Z, *S, *G1, *G2, *F, *E, *G3, *G4, *A, *T;
  float* N;     // explicit noise term, or NULL when the model has none
  int64_t ts;
};
int phase_blocks(int phase, int h, int w, int b);

// The geometry of cube c as wave-uniform (scalar-register) values: the
// table is read once per block and every field is made uniform explicitly,
// so the per-cube sizes and offsets do not occupy vector registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ CubeGeo uniform_geo(const CubeGeo* geo, int c) {
  const CubeGeo g = geo[c];
  CubeGeo u;
  u.h = __builtin_amdgcn_readfirstlane(g.h);
  u.w = __builtin_amdgcn_readfirstlane(g.w);
  u.b = __builtin_amdgcn_readfirstlane(g.b);
  u.nb_w = __builtin_amdgcn_readfirstlane(g.nb_w);
  u.cw_h = __builtin_amdgcn_readfirstlane(g.cw_h);
  u.nb_wi = __builtin_amdgcn_readfirstlane(g.nb_wi);
  u.mm = __builtin_amdgcn_readfirstlane(g.mm);
  u.off = uniform_i64(g.off);
  u.spec_off = uniform_i64(g.spec_off);
  u.slice_base = uniform_i64(g.slice_base);
  return u;
}
// The cube owning block blockIdx.x of a batched launch, and the block's index
// within that cube's own grid.
struct CubeSel {
  int c, bid, nblk;
};
__device__ __forceinline__ CubeSel select_cube(const BatchTab& bt) {
  CubeSel r;
  r.c = __builtin_amdgcn_readfirstlane(find_cube(bt.bstart, bt.nc, blockIdx.x));
  r.bid = blockIdx.x - __builtin_amdgcn_readfirstlane(bt.bstart[r.c]);
  r.nblk = __builtin_amdgcn_readfirstlane(bt.bstart[r.c + 1] - bt.bstart[r.c]);
  return r;
}
// XCD-aware order of a cube's blocks over its column chunks.  Blocks are
// dispatched to the 8 XCDs in turn, so the blocks of one residue class mod 8
// share an XCD and its L2; they take consecutive chunks, and the cache lines
// that two neighbouring chunks share are fetched into one L2 instead of two.
// A bijection of [0, nblk): the chunks bid', bid' + nblk, ... of the returned
// bid' still cover every chunk once.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
  const int c = bid & 7, full = nblk >> 3, rem = nblk & 7;
  return c * full + (c < rem ? c : rem) + (bid >> 3);
}
int geo_rows_nb(int w);
int geo_rows_nb_inv(int w);
int geo_cols_cw(int h);
size_t geo_fft_h_lds(int h);  // dynamic LDS bytes of the h FFT
// dynamic LDS bytes of the DFT-matrix transforms along h, w (forward), w (inverse)
size_t dftmm_lds_h(int h);
size_t dftmm_lds_w(int w);
size_t dftmm_lds_wi(int w);
int dftmm_blocks_h(int h, int w, int b);   // per-cube blocks of the h transform
int dftmm_blocks_w(int h, int w, int b);   // and of the forward w transform
void prepare_fft_h(size_t lds);  // grants that LDS to the h FFT kernels

// One cube's pointers for the adjoint of an iteration (all offset to the
// cube; gradient-shaped arrays are 3 components spaced by ts, the per-cube
// scratch dirE, A by as).  ga* may all be NULL (zero cotangent), gX too.
struct VjpCube {
  int h, w, b;
  int64_t ts, as;
  const float *G4;                      // state before: Gamma4
  const float *S1, *F1;                 // state after: S', F'
  const float *gaZ, *gaS, *gaF, *gaE, *gaG1, *gaG2, *gaG3, *gaG4;
  const float* gX;
  float *gbZ, *gbS, *gbF, *gbE, *gbG1, *gbG2, *gbG3, *gbG4;
  float *gL, *gZp, *gFp;                // cotangent scratch (batch-sized)
  float *dirE, *A;                      // t-SVT direction and point (per cube)
  float* gY;                            // accumulated cotangent of O
  bool initial;                         // the state before has Z = O (gb.Z also flows into gY)
};

void launch_fill(float* p, int64_t n, float v, hipStream_t s);
void launch_copy(float* dst, const float* src, int64_t n, hipStream_t s);
void launch_set_mu(double* mu, double v, hipStream_t s);
void launch_fill_hash(float* p, int64_t n, uint32_t seed, hipStream_t s);
// Per-cube stopping state of an iteration (all device arrays, or halt NULL
// for runs without a stopping test).
struct StopState {
  int* halt;            // [nc] 1 once the cube met the stopping test
  int* iters;           // [nc] iterations the cube has run since the reset
  int* ran;             // [1] set when some cube ran this iteration (read by the mu step)
  const double* eps;    // [1] stopping tolerance, <= 0: no test
};
void launch_finish_iter(const double* part, int n_cubes, const double* mu, double* out, double* res_user,
                        int* flag, const StopState* st, hipStream_t s);
void launch_mu_step(double* mu, double rho, double mu_max, int* ran, hipStream_t s);
void launch_fill_int(int* p, int64_t n, int v, hipStream_t s);
void launch_set_double(double* p, double v, hipStream_t s);
void launch_lrhs_batch(const BatchTab& bt, const BatchPtrs& p, const Weights& wt, const double* mu, hipStream_t s);
void launch_grad_shrink_batch(const BatchTab& bt, const BatchPtrs& p, const Weights& wt, const double* mu,
                              double* part, hipStream_t s);
void launch_rfft_w_batch(const BatchTab& bt, const float* T, float2* spec, hipStream_t s);
void launch_irfft_w_batch(const BatchTab& bt, const float2* spec, float* Z, double* part, hipStream_t s);
void launch_fft_h_batch(const BatchTab& bt, float2* spec, int sign, hipStream_t s);
void launch_tri_b_batch(const BatchTab& bt, float2* spec, const double wts[3], const double* mu, hipStream_t s);
void launch_band_dft_batch(const BatchTab& bt, const float* A, int64_t a_stride, float* slices, hipStream_t s);
void launch_band_idft_batch(const BatchTab& bt, const float* slices, float* E, int64_t e_stride, const float* F,
                            float* G4, const double* mu, double* part, hipStream_t s);

// --- Z-update: FFT along w and h, periodic tridiagonal solve along b -------
// spec holds b * h * (w/2+1) complex values.
void launch_rfft_w(const float* T, float2* spec, int h, int w, int b, hipStream_t s);
void launch_fft_h(float2* spec, int h, int w, int b, int sign, hipStream_t s);
void launch_tri_b(float2* spec, int h, int w, int b, const double wts[3], const double* mu, double mu_host,
                  hipStream_t s);
// Z <- irfft; if part != NULL also writes sum (Z_new - Z_old)^2 partials (slot R_DUAL_Z).
void launch_irfft_w(const float2* spec, float* Z, int h, int w, int b, double* part, hipStream_t s);
// The same transforms as DFT-matrix products (lengths with dft_mm_len); the
// batched forms take the cubes whose CubeGeo::mm bit is set.
void launch_dftmm_rw(const float* T, float2* spec, int h, int w, int b, hipStream_t s);
void launch_dftmm_h(float2* spec, int h, int w, int b, int sign, hipStream_t s);
void launch_dftmm_irw(const float2* spec, float* Z, int h, int w, int b, double* part, hipStream_t s);
void launch_dftmm_rw_batch(const BatchTab& bt, const float* T, float2* spec, hipStream_t s);
void launch_dftmm_h_batch(const BatchTab& bt, float2* spec, int sign, hipStream_t s);
void launch_dftmm_irw_batch(const BatchTab& bt, const float2* spec, float* Z, double* part, hipStream_t s);

// --- band DFT (t-SVT forward) and inverse (+ Gamma4 ascent) ---------------
// A: n_t real cubes spaced by a_stride floats; slices: planar complex,
// [t][k][re|im][h][w] with k < b/2+1.
void launch_band_dft(const float* A, int64_t a_stride, int n_t, float* slices, int h, int w, int b, hipStream_t s);
// E_t = IDFT_b(slices); if G4 != NULL: Gamma4 += mu (E - F) and residual partials (slot R_FRO_EF).
void launch_band_idft(const float* slices, int n_t, float* E, int64_t e_stride, int h, int w, int b,
                      const float* F, float* G4, const double* mu, double* part, hipStream_t s);

// --- slice SVT ------------------------------------------------------------
constexpr int kTriVariants = 5;   // tridiagonalisation shapes (codes 8, 12, 16, 112, 108)
constexpr int kTriDefault = 3;   // 112: register tiles, 12 waves (the tuned shape at 256 x 256)
constexpr int kTriSmallN = 128;  // slices up to this n take the 4-wave register-tile block
int tri_variant_code(int v);      // 100 kind + waves
bool tri_variant_onchip(int v, int n);
// thresh: t = alpha / mu read on the device (mu != NULL) or the fixed value.
struct SvtLaunch {
  const SliceDesc* desc;   // device array [n_slices]
  int n_slices;
  int max_n1, max_m1;      // over slices
  int min_n1 = 0;          // over slices (0: not known)
  float* slices;           // base of the slice planes (input M, output E_hat)
  float2* gram;            // packed Grams / reflectors
  float* V;                // eigenvectors (planar)
  float* B;                // back-projection intermediate
  double* tri;             // tridiagonal scratch
  double* xs;              // eigenvector scratch
  float* fval;             // shrink factors
  float* Twy;              // T factors of the blocked back-transform
  int* rcount;             // surviving singular values per slice
  const double* mu;        // device mu or NULL
  double alpha;            // threshold numerator (t = alpha / mu) when mu != NULL
  float thresh;            // fixed threshold when mu == NULL
  int precision;
  int tri_variant = kTriDefault;  // tridiagonalisation shape (autotuned)
  const int* halt = nullptr;      // device [cubes] or NULL: slices of halted cubes are skipped
};
// Slices beyond the last full round of the one-block-per-slice kernels run
// on a second stream from the tridiagonalisation on, after the first group's
// tridiagonalisation, so that they overlap the first group's later stages
// instead of occupying a few compute units while the rest wait.
struct SvtSplit {
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t big = nullptr;   // the first group's slices above kTriSmallN reduced (on s2)
  int first = 0;   // slices [0, first) on the main stream, the rest on s2; 0: no split
};
// The first group's size for n_slices slices (0: no split), from the
// device's compute-unit count.
int svt_split_point(int n_slices);
void launch_svt(const SvtLaunch& L, hipStream_t s, StageTimer* tm = nullptr, const SvtSplit* sp = nullptr);
// Single stages of launch_svt (the autotuner times them in isolation).
void launch_svt_gram(const SvtLaunch& L, hipStream_t s);
void launch_svt_tridiag(const SvtLaunch& L, hipStream_t s, int which = 3);
// Host-side kernel attributes for slices up to max_n1 (call before capture).
void prepare_svt(int max_n1);

// Derivative of the slice SVT at the slices of fw.slices along the
// direction slices dsl (same layout); the result replaces dsl.  fw.fval
// receives the shrink factors g, acon the per-column threshold-derivative
// terms (already weighted by the slice's Fourier weight and 1/mu).
struct SvtVjpLaunch {
  SvtLaunch fw;
  float* dsl;      // direction slices in, derivative slices out
  float* C;        // D V (B-sized)
  float* R;        // B W + C diag(g) (B-sized)
  float* W;        // g1 o H, r x r per slice (V-sized)
  float* sig;      // singular values (fval-sized)
  const float* ones;  // fval-sized, every entry 1
  double* acon;    // fval-sized
};
void launch_svt_vjp(const SvtVjpLaunch& J, hipStream_t s);

// --- truncated-Tucker L-update (k_tucker.hip) -----------------------------
// Launch kinds of the HOOI phases; block ranges per cube in TkTab.bstart.
enum TkKind { TK_GRAM0 = 0, TK_GRAM1, TK_GRAM2, TK_RED0, TK_RED1, TK_RED2, TK_PROJ0, TK_PROJ1, TK_PROJ2,
              TK_PROD0, TK_PROD1, TK_PROD2, TK_KINDS };
struct TkGeo {
  int h, w, b;
  int groups[3];          // contraction groups of the mode Grams
  int64_t kg[3];          // contraction length per group (multiple of 32)
  int64_t off;            // element offset of the cube in the packed batch
  int64_t p_off[3];       // float offsets of the mode projectors (d x d)
  int64_t part_off[3];    // float offsets of the Gram partials [tile][group][64][64]
};
struct TkTab {
  const TkGeo* geo;       // device [nc]
  const int* bstart;      // device [TK_KINDS][nc + 1]
  int nc;
  int nblocks[TK_KINDS];
  const int* halt;        // device [nc] or NULL: halted cubes are skipped
  __host__ __device__ int kind_off(int k) const { return k * (nc + 1); }
};
void launch_tk_gram(const TkTab& tab, int M, const float* X, float* part, hipStream_t s);
void launch_tk_reduce(const TkTab& tab, int M, const float* part, float2* gram, const SliceDesc* hdesc,
                      hipStream_t s);
void launch_tk_proj(const TkTab& tab, int M, const SliceDesc* hdesc, const float* V, const int* rcount, float* P,
                    hipStream_t s);
void launch_tk_prod(const TkTab& tab, int M, const float* X, const float* P, float* Y, float* L, float* T,
                    const double* mu, bool fin, hipStream_t s);
// Leading eigenpairs of the slices' packed Hermitian matrices: the SVT's
// tridiagonalisation, eigenvalue, eigenvector and back-transform stages with
// every slice keeping its SliceDesc::keep largest eigenpairs (V columns).
void launch_sym_eig(const SvtLaunch& L, hipStream_t s);

// --- adjoint of one iteration (k_vjp.hip) ---------------------------------
void launch_vjp_post(const VjpCube& c, const double* mu, double* part_lam, hipStream_t s);
void launch_vjp_shrinkf(const VjpCube& c, const float* gA, const double* mu, double* part_tau, hipStream_t s);
void launch_vjp_divt(const VjpCube& c, float* T, const double w[3], hipStream_t s);
void launch_vjp_pre(const VjpCube& c, const float* gT, const double w[3], const double* mu, hipStream_t s);
// gw[c] += (tau, alpha, lambda) cotangents; part [n_cubes][2][LRSTV_PARTS]
// (tau, lambda block partials), acon_range [n_cubes][2] index ranges of acon.
void launch_vjp_finish(const double* part, const double* acon, const int64_t* acon_range, int n_cubes, double* gw,
                       hipStream_t s);
// out[c] = sum of acon over acon_range[c]
void launch_sum_ranges(const double* acon, const int64_t* range, int n, double* out, hipStream_t s);

}  // namespace lrstv
