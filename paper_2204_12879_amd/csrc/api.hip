// C ABI of the LRSTV library (declared in include/lrstv.h): argument checks,
// workspace carve-up, slice tables and the per-iteration launch schedule of
// Algorithm 1 (Sec. III-C).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lrstv.h"
#include "common.hpp"

static_assert(LRSTV_MAX_SIDE == LRSTV_MAX_SIDE_DEV, "device-side size bound out of step");
#include "kernels.hpp"
static_assert(lrstv::kTriVariants <= LRSTV_MAX_TRI_SHAPES, "tuning record too small for the shape table");

using namespace lrstv;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(LRSTV_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ workspace ---
namespace {

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct CubeInfo {
  int h, w, b, s;
  int64_t off;         // element offset in the packed batch
  int64_t spec_off;    // complex offset of the half spectrum (Z-solve scratch)
  int64_t slice0;      // index of the first slice of this cube
  int64_t slice_base;  // float offset of this cube's slices
};

// Slice tables and per-slice scratch sizes for a list of cubes with `nt`
// tensors each.
struct SliceLayout {
  std::vector<SliceDesc> desc;
  int64_t slices_floats = 0, gram_c = 0, v_floats = 0, b_floats = 0, tri_d = 0, xs_d = 0, f_floats = 0,
          wy_floats = 0;
  int max_n1 = 0, max_m1 = 0;
  int min_n1 = 0;   // 0 until a slice is added
};

// T factors of the blocked back-transform: one 64 x 64 complex block per 64
// reflectors (planar re / im).
int64_t wy_block_floats(int n1) { return (int64_t)((n1 - 1 + 63) / 64) * 64 * 64 * 2; }

SliceLayout make_slices(std::vector<CubeInfo>& cubes, int nt) {
  SliceLayout L;
  for (size_t c = 0; c < cubes.size(); ++c) {
    CubeInfo& ci = cubes[c];
    const int h = ci.h, w = ci.w, s = ci.s;
    const int64_t hw = (int64_t)h * w;
    const int n1 = h < w ? h : w, m1 = h < w ? w : h;
    ci.slice0 = (int64_t)L.desc.size();
    ci.slice_base = L.slices_floats;
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < s; ++k) {
        SliceDesc d;
        d.h = h;
        d.w = w;
        d.n1 = n1;
        d.m1 = m1;
        d.tall = h >= w;
        d.cube = (int)c;
        d.fw = (float)((k == 0 || 2 * k == ci.b) ? 1 : 2) / (float)ci.b;
        d.a_off = L.slices_floats + ((int64_t)t * s + k) * 2 * hw;
        d.g_off = L.gram_c;
        d.v_off = L.v_floats;
        d.b_off = L.b_floats;
        d.t_off = L.tri_d;
        d.x_off = L.xs_d;
        d.f_off = L.f_floats;
        d.y_off = L.wy_floats;
        d.keep = 0;
        d.prio = 0;
        L.gram_c += (int64_t)n1 * (n1 + 1) / 2;
        L.v_floats += 2 * (int64_t)n1 * n1;
        L.b_floats += 2 * hw;
        L.tri_d += 6 * (int64_t)n1;
        L.xs_d += 3 * (int64_t)n1 * n1;
        L.f_floats += n1;
        L.wy_floats += wy_block_floats(n1);
        L.desc.push_back(d);
      }
    L.slices_floats += (int64_t)nt * s * 2 * hw;
    if (n1 > L.max_n1) L.max_n1 = n1;
    if (L.min_n1 == 0 || n1 < L.min_n1) L.min_n1 = n1;
    if (m1 > L.max_m1) L.max_m1 = m1;
  }
  return L;
}

}  // namespace

struct lrstv_handle_s {
  std::vector<CubeInfo> cubes;
  int64_t total = 0, nmax = 0, specmax = 0, spec_total = 0;
  lrstv_params par;
  hipStream_t stream;
  SliceLayout sl;
  // state
  float *O, *L, *Z, *S, *G1, *G2, *F, *E, *G3, *G4, *N;
  // scratch
  float *T, *A, *slices, *V, *B, *fval, *Twy;
  float2 *spec, *gram;
  double *tri, *xs, *mu, *part, *res_last;
  int *rcount, *flag;
  // on-device stopping test (Algorithm 1's convergence check)
  int *halt, *iters, *ran;
  double* eps;
  int* poll_host = nullptr;          // pinned [2][nc + 1]: halt flags and the non-finite flag
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  SliceDesc* desc;
  CubeGeo* geo;        // device [n_cubes]
  int* bstart;         // device [PH_COUNT][n_cubes + 1]
  BatchTab bt[PH_COUNT];
  int tri_variant = kTriDefault;   // tridiagonalisation shape (lrstv_autotune / lrstv_set_tuning)
  StageTimer timer;
  // per-cube index ranges of the per-column t-SVT threshold terms (adjoint)
  std::vector<int64_t> acon_range;
  // hipGraph replay of one iteration (lrstv_set_graph)
  bool graph_on = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // second stream of the slice SVT (the slices beyond the last full round)
  SvtSplit split;
  // truncated-Tucker L-update (HOOI): eigen-slices [mode][cube], projectors,
  // Gram partials and the launch tables
  bool tk_on = false;
  bool tk_mode[3] = {false, false, false};   // some cube truncates this mode
  SliceLayout tsl;
  SliceDesc* tdesc = nullptr;
  float2* tgram = nullptr;
  float *tV = nullptr, *tTwy = nullptr, *tP = nullptr, *tpart = nullptr;
  double *ttri = nullptr, *txs = nullptr;
  int* trcount = nullptr;
  TkGeo* tgeo = nullptr;
  int* tbstart = nullptr;
  TkTab ttab;
  std::vector<TkGeo> tgeo_h;
  std::vector<int> tbstart_h;
  int64_t tp_total = 0, tpart_total = 0;
  // Non-finite latch: k_finish_iter sets *flag; after every lrstv_iterate
  // the flag is copied to pinned host memory asynchronously and the copy
  // marked by flag_ev, so that a later call can see it without a sync.
  int* flag_host = nullptr;
  hipEvent_t flag_ev = nullptr;
  bool flag_pending = false;   // a copy has been enqueued since the last reset
  bool flag_known = false;     // a completed copy read 1
  ~lrstv_handle_s() {
    for (hipEvent_t e : poll_ev)
      if (e) (void)hipEventDestroy(e);
    if (poll_host) (void)hipHostFree(poll_host);
    if (flag_ev) (void)hipEventDestroy(flag_ev);
    if (flag_host) (void)hipHostFree(flag_host);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (split.fork) (void)hipEventDestroy(split.fork);
    if (split.join) (void)hipEventDestroy(split.join);
    if (split.big) (void)hipEventDestroy(split.big);
    if (split.s2) (void)hipStreamDestroy(split.s2);
  }
};

static int check_params(const lrstv_params* p) {
  if (!p) return fail(LRSTV_ERR_INVALID_ARG, "params is NULL");
  if (!(p->tau >= 0) || !(p->alpha >= 0) || !(p->lambda >= 0))
    return fail(LRSTV_ERR_INVALID_ARG, "tau, alpha, lambda must be >= 0");
  for (int i = 0; i < 3; ++i)
    if (!(p->w[i] >= 0)) return fail(LRSTV_ERR_INVALID_ARG, "difference weights must be >= 0");
  if (!(p->mu0 > 0)) return fail(LRSTV_ERR_INVALID_ARG, "mu0 must be > 0");
  if (!(p->rho >= 1)) return fail(LRSTV_ERR_INVALID_ARG, "rho must be >= 1");
  if (!(p->mu_max >= p->mu0)) return fail(LRSTV_ERR_INVALID_ARG, "mu_max must be >= mu0");
  if (p->precision != LRSTV_FP32 && p->precision != LRSTV_SPLIT_BF16)
    return fail(LRSTV_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->tv != LRSTV_TV_ANISO && p->tv != LRSTV_TV_ISO)
    return fail(LRSTV_ERR_INVALID_ARG, "unknown gradient term %d", p->tv);
  if (!(p->beta >= 0) || !isfinite(p->beta)) return fail(LRSTV_ERR_INVALID_ARG, "beta must be finite and >= 0");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(p->tucker[i])) return fail(LRSTV_ERR_INVALID_ARG, "Tucker rank fractions must be finite");
  if (p->hooi_sweeps < 0 || p->hooi_sweeps > 100) return fail(LRSTV_ERR_INVALID_ARG, "hooi_sweeps must be in [0, 100]");
  return LRSTV_OK;
}

static int check_dims(int h, int w, int b) {
  if (h < 1 || w < 1 || b < 1) return fail(LRSTV_ERR_INVALID_ARG, "sizes must be >= 1 (got h=%d w=%d b=%d)", h, w, b);
  if (h > LRSTV_MAX_SIDE || w > LRSTV_MAX_SIDE || b > LRSTV_MAX_SIDE)
    return fail(LRSTV_ERR_UNSUPPORTED, "side above %d (h=%d w=%d b=%d)", LRSTV_MAX_SIDE, h, w, b);
  return LRSTV_OK;
}

static int build_cubes(const lrstv_problem* prob, std::vector<CubeInfo>& cubes, int64_t& total, int64_t& nmax,
                       int64_t& specmax, int64_t& spec_total) {
  if (!prob || prob->n_cubes < 1 || !prob->h || !prob->w || !prob->b)
    return fail(LRSTV_ERR_INVALID_ARG, "problem must list n_cubes >= 1 with h, w, b arrays");
  cubes.clear();
  total = 0;
  nmax = 0;
  specmax = 0;
  spec_total = 0;
  for (int c = 0; c < prob->n_cubes; ++c) {
    const int h = prob->h[c], w = prob->w[c], b = prob->b[c];
    int rc = check_dims(h, w, b);
    if (rc) return rc;
    CubeInfo ci;
    ci.h = h;
    ci.w = w;
    ci.b = b;
    ci.s = b / 2 + 1;
    ci.off = total;
    const int64_t N = (int64_t)h * w * b;
    total += N;
    if (N > nmax) nmax = N;
    const int64_t sp = (int64_t)b * h * (w / 2 + 1);
    if (sp > specmax) specmax = sp;
    ci.spec_off = spec_total;
    spec_total += sp;
    cubes.push_back(ci);
  }
  return LRSTV_OK;
}

// Tucker rank of one mode: floor(f d + 1/2) clipped to [1, d]; d when the
// fraction asks for no truncation.
static int tucker_rank(double f, int d) {
  if (!(f > 0.0) || f >= 1.0) return d;
  int r = (int)floor(f * d + 0.5);
  return r < 1 ? 1 : (r > d ? d : r);
}

// The HOOI eigen-slices (one per cube and mode, laid out [mode][cube]; a
// mode a cube keeps at full rank gets no Gram and an identity projector),
// the per-cube launch tables and the projector / partial sizes.  Sets
// H->tk_on when some cube truncates some mode.
static void plan_tucker(lrstv_handle_s* H) {
  const int nc = (int)H->cubes.size();
  H->tk_on = false;
  for (int m = 0; m < 3; ++m) H->tk_mode[m] = false;
  H->tgeo_h.assign(nc, TkGeo());
  H->tbstart_h.assign((size_t)TK_KINDS * (nc + 1), 0);
  for (int c = 0; c < nc; ++c) {
    const CubeInfo& ci = H->cubes[c];
    const int d[3] = {ci.h, ci.w, ci.b};
    for (int m = 0; m < 3; ++m)
      if (tucker_rank(H->par.tucker[m], d[m]) < d[m]) H->tk_mode[m] = H->tk_on = true;
  }
  H->tsl = SliceLayout();
  H->tp_total = H->tpart_total = 0;
  if (!H->tk_on) return;
  SliceLayout& L = H->tsl;
  for (int m = 0; m < 3; ++m)
    for (int c = 0; c < nc; ++c) {
      const CubeInfo& ci = H->cubes[c];
      const int d[3] = {ci.h, ci.w, ci.b};
      const int n = d[m];
      SliceDesc sd;
      memset(&sd, 0, sizeof sd);
      sd.h = sd.w = sd.n1 = sd.m1 = n;
      sd.tall = 1;
      sd.cube = c;
      sd.fw = 1.f;
      sd.g_off = L.gram_c;
      sd.v_off = L.v_floats;
      sd.t_off = L.tri_d;
      sd.x_off = L.xs_d;
      sd.y_off = L.wy_floats;
      sd.keep = tucker_rank(H->par.tucker[m], n);
      L.gram_c += (int64_t)n * (n + 1) / 2;
      L.v_floats += 2 * (int64_t)n * n;
      L.tri_d += 6 * (int64_t)n;
      L.xs_d += 3 * (int64_t)n * n;
      L.wy_floats += wy_block_floats(n);
      L.desc.push_back(sd);
      if (n > L.max_n1) L.max_n1 = n;
      if (L.min_n1 == 0 || n < L.min_n1) L.min_n1 = n;
      if (n > L.max_m1) L.max_m1 = n;
    }
  for (int c = 0; c < nc; ++c) {
    const CubeInfo& ci = H->cubes[c];
    TkGeo& g = H->tgeo_h[c];
    g.h = ci.h;
    g.w = ci.w;
    g.b = ci.b;
    g.off = ci.off;
    const int d[3] = {ci.h, ci.w, ci.b};
    const int64_t K[3] = {(int64_t)ci.b * ci.w, (int64_t)ci.b * ci.h, (int64_t)ci.h * ci.w};
    int nb[TK_KINDS];
    for (int m = 0; m < 3; ++m) {
      const int T = (d[m] + 63) / 64, ntile = T * (T + 1) / 2;
      const bool trunc = tucker_rank(H->par.tucker[m], d[m]) < d[m];
      // about 512 blocks per mode Gram: groups of the contraction, 32-multiples
      int G = (512 + ntile - 1) / ntile;
      int64_t kg = (K[m] + G - 1) / G;
      kg = (kg + 31) / 32 * 32;
      G = (int)((K[m] + kg - 1) / kg);
      g.groups[m] = G;
      g.kg[m] = kg;
      g.p_off[m] = H->tp_total;
      H->tp_total += (int64_t)d[m] * d[m];
      g.part_off[m] = H->tpart_total;
      if (trunc) H->tpart_total += (int64_t)ntile * G * 64 * 64;
      nb[TK_GRAM0 + m] = trunc ? ntile * G : 0;
      nb[TK_RED0 + m] = trunc ? (int)(((int64_t)d[m] * (d[m] + 1) / 2 + 255) / 256) : 0;
      nb[TK_PROJ0 + m] = trunc ? T * T : 0;
    }
    const int TH = (ci.h + 63) / 64, TW = (ci.w + 63) / 64, TB = (ci.b + 63) / 64;
    const int TN = (int)(((int64_t)ci.h * ci.w + 63) / 64);
    nb[TK_PROD0] = ci.b * TH * TW;
    nb[TK_PROD1] = ci.b * TH * TW;
    nb[TK_PROD2] = TB * TN;
    for (int k = 0; k < TK_KINDS; ++k)
      H->tbstart_h[(size_t)k * (nc + 1) + c + 1] = H->tbstart_h[(size_t)k * (nc + 1) + c] + nb[k];
  }
}

static void carve_handle(lrstv_handle_s* H, void* base, size_t* used) {
  Carve cv(base);
  const int64_t T = H->total, nc = (int64_t)H->cubes.size();
  H->O = cv.take<float>(T);
  H->L = cv.take<float>(T);
  H->Z = cv.take<float>(T);
  H->S = cv.take<float>(T);
  H->G1 = cv.take<float>(T);
  H->G2 = cv.take<float>(T);
  H->F = cv.take<float>(3 * T);
  H->E = cv.take<float>(3 * T);
  H->G3 = cv.take<float>(3 * T);
  H->G4 = cv.take<float>(3 * T);
  H->N = cv.take<float>(T);
  H->T = cv.take<float>(T);
  H->A = cv.take<float>(3 * T);
  H->spec = cv.take<float2>(H->spec_total);
  H->slices = cv.take<float>(H->sl.slices_floats);
  H->gram = cv.take<float2>(H->sl.gram_c);
  H->V = cv.take<float>(H->sl.v_floats);
  H->B = cv.take<float>(H->sl.b_floats);
  H->tri = cv.take<double>(H->sl.tri_d);
  H->xs = cv.take<double>(H->sl.xs_d);
  H->Twy = cv.take<float>(H->sl.wy_floats);
  H->fval = cv.take<float>(H->sl.f_floats);
  H->rcount = cv.take<int>(H->sl.desc.size());
  H->desc = cv.take<SliceDesc>(H->sl.desc.size());
  H->geo = cv.take<CubeGeo>(nc);
  H->bstart = cv.take<int>(PH_COUNT * (nc + 1));
  H->mu = cv.take<double>(1);
  H->part = cv.take<double>(nc * R_COUNT * LRSTV_PARTS);
  H->res_last = cv.take<double>(nc * R_COUNT);
  H->flag = cv.take<int>(1);
  if (H->tk_on) {
    const SliceLayout& L = H->tsl;
    H->tdesc = cv.take<SliceDesc>(L.desc.size());
    H->tgram = cv.take<float2>(L.gram_c);
    H->tV = cv.take<float>(L.v_floats);
    H->ttri = cv.take<double>(L.tri_d);
    H->txs = cv.take<double>(L.xs_d);
    H->tTwy = cv.take<float>(L.wy_floats);
    H->trcount = cv.take<int>(L.desc.size());
    H->tP = cv.take<float>(H->tp_total);
    H->tpart = cv.take<float>(H->tpart_total);
    H->tgeo = cv.take<TkGeo>(nc);
    H->tbstart = cv.take<int>((int64_t)TK_KINDS * (nc + 1));
  }
  H->halt = cv.take<int>(nc);
  H->iters = cv.take<int>(nc);
  H->ran = cv.take<int>(1);
  H->eps = cv.take<double>(1);
  *used = cv.off + 256;
}

extern "C" int lrstv_workspace_size(const lrstv_problem* prob, const lrstv_params* par, size_t* bytes) {
  if (!bytes) return fail(LRSTV_ERR_INVALID_ARG, "bytes is NULL");
  int rc = check_params(par);
  if (rc) return rc;
  lrstv_handle_s H;
  rc = build_cubes(prob, H.cubes, H.total, H.nmax, H.specmax, H.spec_total);
  if (rc) return rc;
  H.sl = make_slices(H.cubes, 3);
  H.par = *par;
  plan_tucker(&H);
  carve_handle(&H, nullptr, bytes);
  return LRSTV_OK;
}

extern "C" int lrstv_create(lrstv_handle* out, const lrstv_problem* prob, const lrstv_params* par, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!out) return fail(LRSTV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_params(par);
  if (rc) return rc;
  if (!workspace) return fail(LRSTV_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(LRSTV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  lrstv_handle_s* H = new (std::nothrow) lrstv_handle_s();
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "out of host memory");
  rc = build_cubes(prob, H->cubes, H->total, H->nmax, H->specmax, H->spec_total);
  if (rc) { delete H; return rc; }
  H->par = *par;
  H->stream = (hipStream_t)stream;
  H->timer.s = H->stream;
  H->sl = make_slices(H->cubes, 3);
  plan_tucker(H);
  size_t need = 0;
  carve_handle(H, nullptr, &need);
  if (ws_bytes < need) {
    delete H;
    return fail(LRSTV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  }
  carve_handle(H, workspace, &need);
  // cube geometry and per-phase block ranges of the batched launches
  const int nc = (int)H->cubes.size();
  std::vector<CubeGeo> geo(nc);
  std::vector<int> bstart((size_t)PH_COUNT * (nc + 1), 0);
  size_t lds_w = 0, lds_h = 0, lds_wi = 0, lds_mm_h = 0, lds_mm_w = 0, lds_mm_wi = 0;
  int max_b = 0, reg_h_mask = 0, stockham_h = 0, reg_w_mask = 0, stockham_w = 0, mm_h = 0, mm_w = 0;
  for (int c = 0; c < nc; ++c) {
    const CubeInfo& ci = H->cubes[c];
    CubeGeo& g = geo[c];
    g.h = ci.h;
    g.w = ci.w;
    g.b = ci.b;
    g.nb_w = geo_rows_nb(ci.w);
    g.nb_wi = geo_rows_nb_inv(ci.w);
    g.cw_h = geo_cols_cw(ci.h);
    g.off = ci.off;
    g.spec_off = ci.spec_off;
    g.slice_base = ci.slice_base;
    const size_t lw = (size_t)(2 * g.nb_w + 1) * ci.w * sizeof(float2);
    const size_t lwi = (size_t)(2 * g.nb_wi + 1) * ci.w * sizeof(float2);
    if (lwi > lds_wi) lds_wi = lwi;
    const size_t lh = geo_fft_h_lds(ci.h);
    if (lw > lds_w) lds_w = lw;
    if (lh > lds_h) lds_h = lh;
    if (ci.b > max_b) max_b = ci.b;
    const bool mh = dft_mm_len(ci.h, kMmMaxH), mw = dft_mm_len(ci.w, kMmMaxW);
    g.mm = (mh ? 1 : 0) | (mw ? 2 : 0);
    reg_h_mask |= fft_h_reg_bit(ci.h);
    reg_w_mask |= fft_h_reg_bit(ci.w);
    if (mh) {
      mm_h = 1;
      if (dftmm_lds_h(ci.h) > lds_mm_h) lds_mm_h = dftmm_lds_h(ci.h);
    } else if (fft_h_reg_bit(ci.h) == 0) {
      stockham_h = 1;
    }
    if (mw) {
      mm_w = 1;
      if (dftmm_lds_w(ci.w) > lds_mm_w) lds_mm_w = dftmm_lds_w(ci.w);
      if (dftmm_lds_wi(ci.w) > lds_mm_wi) lds_mm_wi = dftmm_lds_wi(ci.w);
    } else if (fft_h_reg_bit(ci.w) == 0) {
      stockham_w = 1;
    }
    for (int ph = 0; ph < PH_COUNT; ++ph)
      bstart[(size_t)ph * (nc + 1) + c + 1] = bstart[(size_t)ph * (nc + 1) + c] + phase_blocks(ph, ci.h, ci.w, ci.b);
  }
  for (int ph = 0; ph < PH_COUNT; ++ph) {
    BatchTab& bt = H->bt[ph];
    bt.geo = H->geo;
    bt.bstart = H->bstart + (size_t)ph * (nc + 1);
    bt.nc = nc;
    bt.nblocks = bstart[(size_t)ph * (nc + 1) + nc];
    bt.lds_w = lds_w;
    bt.lds_wi = lds_wi;
    bt.lds_h = lds_h;
    bt.max_b = max_b;
    bt.reg_h_mask = reg_h_mask;
    bt.stockham_h = stockham_h;
    bt.reg_w_mask = reg_w_mask;
    bt.stockham_w = stockham_w;
    bt.mm_h = mm_h;
    bt.mm_w = mm_w;
    bt.lds_mm_h = lds_mm_h;
    bt.lds_mm_w = lds_mm_w;
    bt.lds_mm_wi = lds_mm_wi;
    bt.halt = H->halt;
  }
  // slices beyond the last full round of compute units run their later
  // stages beside the first group's (see the split below)
  {
    const int first = svt_split_point((int)H->sl.desc.size());
    for (size_t i = first > 0 ? (size_t)first : H->sl.desc.size(); i < H->sl.desc.size(); ++i) H->sl.desc[i].prio = 1;
  }
  hipError_t e = hipMemcpyAsync(H->desc, H->sl.desc.data(), H->sl.desc.size() * sizeof(SliceDesc),
                                hipMemcpyHostToDevice, H->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(H->geo, geo.data(), geo.size() * sizeof(CubeGeo), hipMemcpyHostToDevice, H->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(H->bstart, bstart.data(), bstart.size() * sizeof(int), hipMemcpyHostToDevice, H->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(H->stream);
  if (e != hipSuccess) {
    delete H;
    return fail(LRSTV_ERR_HIP, "copying the slice table: %s", hipGetErrorString(e));
  }
  if (e == hipSuccess && H->tk_on) {
    // HOOI tables, eigen-slice descriptors, zero Grams (modes kept at full
    // rank are never written) and identity projectors (overwritten each
    // iteration for the truncated modes)
    e = hipMemcpyAsync(H->tdesc, H->tsl.desc.data(), H->tsl.desc.size() * sizeof(SliceDesc),
                       hipMemcpyHostToDevice, H->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(H->tgeo, H->tgeo_h.data(), nc * sizeof(TkGeo), hipMemcpyHostToDevice, H->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(H->tbstart, H->tbstart_h.data(), H->tbstart_h.size() * sizeof(int), hipMemcpyHostToDevice,
                         H->stream);
    std::vector<float> eye((size_t)H->tp_total, 0.f);
    for (int c = 0; c < nc; ++c) {
      const CubeInfo& ci = H->cubes[c];
      const int d[3] = {ci.h, ci.w, ci.b};
      for (int m = 0; m < 3; ++m)
        for (int i = 0; i < d[m]; ++i) eye[(size_t)H->tgeo_h[c].p_off[m] + (size_t)i * d[m] + i] = 1.f;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(H->tP, eye.data(), eye.size() * sizeof(float), hipMemcpyHostToDevice, H->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(H->stream);
    launch_fill((float*)H->tgram, 2 * H->tsl.gram_c, 0.f, H->stream);
    H->ttab.geo = H->tgeo;
    H->ttab.bstart = H->tbstart;
    H->ttab.nc = nc;
    H->ttab.halt = H->halt;
    for (int k = 0; k < TK_KINDS; ++k) H->ttab.nblocks[k] = H->tbstart_h[(size_t)k * (nc + 1) + nc];
    if (e != hipSuccess) {
      delete H;
      return fail(LRSTV_ERR_HIP, "copying the Tucker tables: %s", hipGetErrorString(e));
    }
  }
  prepare_svt(H->tk_on && H->tsl.max_n1 > H->sl.max_n1 ? H->tsl.max_n1 : H->sl.max_n1);
  prepare_fft_h(lds_h);
  H->split.first = svt_split_point((int)H->sl.desc.size());
  if (H->split.first > 0) {
    e = hipStreamCreateWithFlags(&H->split.s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&H->split.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&H->split.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&H->split.big, hipEventDisableTiming);
    if (e != hipSuccess) {
      delete H;
      return fail(LRSTV_ERR_HIP, "creating the second stream: %s", hipGetErrorString(e));
    }
  }
  e = hipHostMalloc((void**)&H->flag_host, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&H->flag_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&H->poll_host, 2 * (size_t)(nc + 1) * sizeof(int), hipHostMallocDefault);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&H->poll_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    delete H;
    return fail(LRSTV_ERR_HIP, "creating the non-finite latch: %s", hipGetErrorString(e));
  }
  *H->flag_host = 0;
  launch_fill_int(H->flag, 1, 0, H->stream);
  launch_fill_int(H->halt, nc, 0, H->stream);
  launch_fill_int(H->iters, nc, 0, H->stream);
  launch_fill_int(H->ran, 1, 0, H->stream);
  launch_set_double(H->eps, 0.0, H->stream);
  launch_set_mu(H->mu, par->mu0, H->stream);
  *out = H;
  return LRSTV_OK;
}

// True when a completed copy of the device latch has shown a non-finite
// residual since the last reset (no synchronisation).
static bool nonfinite_seen(lrstv_handle_s* H) {
  if (H->flag_pending && hipEventQuery(H->flag_ev) == hipSuccess) {
    H->flag_pending = false;
    H->flag_known = H->flag_known || *H->flag_host != 0;
  }
  return H->flag_known;
}

// Enqueue the copy of the device latch behind the work already queued.
static int post_flag_copy(lrstv_handle_s* H) {
  HIPCHK(hipMemcpyAsync(H->flag_host, H->flag, sizeof(int), hipMemcpyDeviceToHost, H->stream));
  HIPCHK(hipEventRecord(H->flag_ev, H->stream));
  H->flag_pending = true;
  return LRSTV_OK;
}

extern "C" void lrstv_destroy(lrstv_handle hd) { delete hd; }

extern "C" int lrstv_reset(lrstv_handle H, const float* Y) {
  if (!H || !Y) return fail(LRSTV_ERR_INVALID_ARG, "handle or Y is NULL");
  const int64_t T = H->total;
  hipStream_t s = H->stream;
  launch_copy(H->O, Y, T, s);
  launch_copy(H->Z, Y, T, s);
  launch_copy(H->L, Y, T, s);
  launch_fill(H->S, T, 0.f, s);
  launch_fill(H->G1, T, 0.f, s);
  launch_fill(H->G2, T, 0.f, s);
  launch_fill(H->F, 3 * T, 0.f, s);
  launch_fill(H->E, 3 * T, 0.f, s);
  launch_fill(H->G3, 3 * T, 0.f, s);
  launch_fill(H->G4, 3 * T, 0.f, s);
  launch_fill(H->N, T, 0.f, s);
  launch_set_mu(H->mu, H->par.mu0, s);
  launch_fill_int(H->flag, 1, 0, s);
  // stopping state: no cube halted, no test until lrstv_solve sets eps
  const int nc = (int)H->cubes.size();
  launch_fill_int(H->halt, nc, 0, s);
  launch_fill_int(H->iters, nc, 0, s);
  launch_fill_int(H->ran, 1, 0, s);
  launch_set_double(H->eps, 0.0, s);
  // copies enqueued before this reset are no longer looked at: the next
  // lrstv_iterate enqueues a copy behind them and re-records the event
  H->flag_pending = false;
  H->flag_known = false;
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

static BatchPtrs batch_ptrs(lrstv_handle_s* H) {
  BatchPtrs p;
  p.O = H->O;
  p.L = H->L;
  p.Z = H->Z;
  p.S = H->S;
  p.G1 = H->G1;
  p.G2 = H->G2;
  p.F = H->F;
  p.E = H->E;
  p.G3 = H->G3;
  p.G4 = H->G4;
  p.A = H->A;
  p.T = H->T;
  p.N = H->par.beta > 0 ? H->N : nullptr;
  p.ts = H->total;
  return p;
}

// The eigen-solves of the HOOI slices of `mode` (0, 1, 2), or of all three
// modes (mode < 0).
static void tucker_eig(lrstv_handle_s* H, int mode, hipStream_t s) {
  const int nc = (int)H->cubes.size();
  SvtLaunch L;
  L.desc = H->tdesc + (mode < 0 ? 0 : mode * nc);
  L.n_slices = mode < 0 ? 3 * nc : nc;
  L.max_n1 = H->tsl.max_n1;
  L.min_n1 = H->tsl.min_n1;
  L.max_m1 = H->tsl.max_m1;
  L.slices = nullptr;
  L.gram = H->tgram;
  L.V = H->tV;
  L.B = nullptr;
  L.tri = H->ttri;
  L.xs = H->txs;
  L.Twy = H->tTwy;
  L.fval = nullptr;
  L.rcount = H->trcount + (mode < 0 ? 0 : mode * nc);
  L.mu = nullptr;
  L.alpha = 0.0;
  L.thresh = -1.f;
  L.precision = LRSTV_FP32;
  L.tri_variant = H->tri_variant;
  L.halt = H->halt;
  launch_sym_eig(L, s);
}

// HOOI of the average the L-update wrote into L (Sec. III-C, eq.
// X_solution): truncated-HOSVD start, H->par.hooi_sweeps sweeps over the
// truncated modes, then L = X x_1 P_1 x_2 P_2 x_3 P_3, the last product
// also moving T_z by mu (L - X).  The t-SVT input buffer A (free until the
// F-update) holds the two intermediate tensors.
static void run_hooi(lrstv_handle_s* H, hipStream_t s) {
  const TkTab& tab = H->ttab;
  float* X = H->L;
  float* t0 = H->A;
  float* t1 = H->A + H->total;
  for (int m = 0; m < 3; ++m) {
    if (!H->tk_mode[m]) continue;
    launch_tk_gram(tab, m, X, H->tpart, s);
    launch_tk_reduce(tab, m, H->tpart, H->tgram, H->tdesc, s);
  }
  tucker_eig(H, -1, s);
  for (int m = 0; m < 3; ++m)
    if (H->tk_mode[m]) launch_tk_proj(tab, m, H->tdesc, H->tV, H->trcount, H->tP, s);
  for (int sw = 0; sw < H->par.hooi_sweeps; ++sw)
    for (int m = 0; m < 3; ++m) {
      if (!H->tk_mode[m]) continue;
      const int a = m == 0 ? 1 : 0, b = m == 2 ? 1 : 2;   // the other two modes, in order
      launch_tk_prod(tab, a, X, H->tP, t0, nullptr, nullptr, nullptr, false, s);
      launch_tk_prod(tab, b, t0, H->tP, t1, nullptr, nullptr, nullptr, false, s);
      launch_tk_gram(tab, m, t1, H->tpart, s);
      launch_tk_reduce(tab, m, H->tpart, H->tgram, H->tdesc, s);
      tucker_eig(H, m, s);
      launch_tk_proj(tab, m, H->tdesc, H->tV, H->trcount, H->tP, s);
    }
  launch_tk_prod(tab, 0, X, H->tP, t0, nullptr, nullptr, nullptr, false, s);
  launch_tk_prod(tab, 1, t0, H->tP, t1, nullptr, nullptr, nullptr, false, s);
  launch_tk_prod(tab, 2, t1, H->tP, nullptr, H->L, H->T, H->mu, true, s);
}

// One iteration over the whole batch: every stencil, FFT and band-transform
// phase is one launch over all cubes (per-cube block ranges), the slice SVT
// one launch per kernel over all slices.
static void run_iteration(lrstv_handle_s* H, double* res_user) {
  hipStream_t s = H->stream;
  StageTimer& tm = H->timer;
  Weights wt;
  wt.tau = H->par.tau;
  wt.alpha = H->par.alpha;
  wt.lam = H->par.lambda;
  for (int i = 0; i < 3; ++i) wt.w[i] = H->par.w[i];
  wt.iso = H->par.tv == LRSTV_TV_ISO;
  wt.beta = H->par.beta;
  const int nc = (int)H->cubes.size();
  const BatchPtrs bp = batch_ptrs(H);
  tm.begin(ST_LRHS);
  launch_lrhs_batch(H->bt[PH_LRHS], bp, wt, H->mu, s);                  // 1st step + T_z
  tm.end(ST_LRHS);
  if (H->tk_on) {                                                       // truncated Tucker ranks
    tm.begin(ST_HOOI);
    run_hooi(H, s);
    tm.end(ST_HOOI);
  }
  tm.begin(ST_RFFT_W);
  launch_rfft_w_batch(H->bt[PH_RFFT_W], H->T, H->spec, s);              // 2nd step: Z solve
  tm.end(ST_RFFT_W);
  tm.begin(ST_FFT_H);
  launch_fft_h_batch(H->bt[PH_FFT_H], H->spec, -1, s);
  tm.end(ST_FFT_H);
  tm.begin(ST_TRI_B);
  launch_tri_b_batch(H->bt[PH_TRI_B], H->spec, wt.w, H->mu, s);
  tm.end(ST_TRI_B);
  tm.begin(ST_FFT_H);
  launch_fft_h_batch(H->bt[PH_FFT_H], H->spec, +1, s);
  tm.end(ST_FFT_H);
  tm.begin(ST_IRFFT_W);
  launch_irfft_w_batch(H->bt[PH_PARTS], H->spec, H->Z, H->part, s);
  tm.end(ST_IRFFT_W);
  // 3rd, 5th and 6th steps (F, S, Gamma1..3); A = F - Gamma4/mu into scratch
  tm.begin(ST_GRAD_SHRINK);
  launch_grad_shrink_batch(H->bt[PH_PARTS], bp, wt, H->mu, H->part, s);
  tm.end(ST_GRAD_SHRINK);
  tm.begin(ST_BAND_DFT);
  launch_band_dft_batch(H->bt[PH_BAND_DFT], H->A, H->total, H->slices, s);
  tm.end(ST_BAND_DFT);
  // 4th step: t-SVT of every Fourier slice of every gradient tensor
  SvtLaunch sv;
  sv.desc = H->desc;
  sv.n_slices = (int)H->sl.desc.size();
  sv.max_n1 = H->sl.max_n1;
  sv.min_n1 = H->sl.min_n1;
  sv.max_m1 = H->sl.max_m1;
  sv.slices = H->slices;
  sv.gram = H->gram;
  sv.V = H->V;
  sv.B = H->B;
  sv.tri = H->tri;
  sv.xs = H->xs;
  sv.Twy = H->Twy;
  sv.fval = H->fval;
  sv.rcount = H->rcount;
  sv.mu = H->mu;
  sv.alpha = H->par.alpha;
  sv.thresh = 0.f;
  sv.precision = H->par.precision;
  sv.tri_variant = H->tri_variant;
  sv.halt = H->halt;
  launch_svt(sv, s, &tm, &H->split);
  tm.begin(ST_BAND_IDFT);
  launch_band_idft_batch(H->bt[PH_PARTS], H->slices, H->E, H->total, H->F, H->G4, H->mu, H->part, s);
  tm.end(ST_BAND_IDFT);
  tm.begin(ST_FINISH);
  StopState stop;
  stop.halt = H->halt;
  stop.iters = H->iters;
  stop.ran = H->ran;
  stop.eps = H->eps;
  launch_finish_iter(H->part, nc, H->mu, H->res_last, res_user, H->flag, &stop, s);   // convergence check
  launch_mu_step(H->mu, H->par.rho, H->par.mu_max, H->ran, s);       // 7th step
  tm.end(ST_FINISH);
}

// Capture one iteration into a graph (once).  Capture runs on a private
// non-blocking stream (the caller's stream may be the legacy null stream,
// which cannot be captured); the graph is then launched on the caller's
// stream.  Every per-iteration scalar (mu, residuals, shrink thresholds)
// lives on the device, so replays need no host work; fills use kernels.
static int ensure_graph(lrstv_handle_s* H) {
  if (H->gexec) return LRSTV_OK;
  hipStream_t cap = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  // work already queued on the caller's stream must not race the capture's
  // (never executed) recording: nothing is launched, only recorded
  const bool timing = H->timer.on;
  hipStream_t user = H->stream;
  H->timer.on = false;
  H->stream = cap;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  hipGraph_t g = nullptr;
  if (e == hipSuccess) {
    run_iteration(H, nullptr);
    e = hipStreamEndCapture(cap, &g);
  }
  H->stream = user;
  H->timer.on = timing;
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LRSTV_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
  }
  H->graph = g;
  HIPCHK(hipGraphInstantiate(&H->gexec, H->graph, nullptr, nullptr, 0));
  return LRSTV_OK;
}

extern "C" int lrstv_set_graph(lrstv_handle H, int32_t enable) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  H->graph_on = enable != 0;
  if (H->graph_on) return ensure_graph(H);
  return LRSTV_OK;
}

extern "C" int lrstv_iterate(lrstv_handle H, int32_t n_iter, double* residuals) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  if (n_iter < 0) return fail(LRSTV_ERR_INVALID_ARG, "n_iter must be >= 0");
  if (nonfinite_seen(H))
    return fail(LRSTV_ERR_NONFINITE, "an earlier iteration met a non-finite residual (latched until reset)");
  const int nc = (int)H->cubes.size();
  if (H->graph_on && !H->timer.on) {
    int rc = ensure_graph(H);
    if (rc) return rc;
    for (int it = 0; it < n_iter; ++it) {
      HIPCHK(hipGraphLaunch(H->gexec, H->stream));
      if (residuals)
        launch_copy((float*)(residuals + (int64_t)it * nc * R_COUNT), (const float*)H->res_last, 2 * nc * R_COUNT,
                    H->stream);
    }
  } else {
    for (int it = 0; it < n_iter; ++it)
      run_iteration(H, residuals ? residuals + (int64_t)it * nc * R_COUNT : nullptr);
  }
  HIPCHK(hipGetLastError());
  return n_iter > 0 ? post_flag_copy(H) : LRSTV_OK;
}

extern "C" int lrstv_check(lrstv_handle H) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  if (H->flag_pending) HIPCHK(hipEventSynchronize(H->flag_ev));
  if (nonfinite_seen(H)) return fail(LRSTV_ERR_NONFINITE, "an iteration met a non-finite residual");
  return LRSTV_OK;
}

extern "C" int lrstv_read_output(lrstv_handle H, float* X, float* S) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  if (nonfinite_seen(H))
    return fail(LRSTV_ERR_NONFINITE, "an earlier iteration met a non-finite residual (latched until reset)");
  if (X) launch_copy(X, H->L, H->total, H->stream);
  if (S) launch_copy(S, H->S, H->total, H->stream);
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

// Iterations per chunk of lrstv_solve with a stopping test: the host looks at
// the halt flags of chunk j - 1 while chunk j is queued, so the device never
// waits for the host, and at most two chunks run after every cube has halted
// (their kernels return at once for halted cubes).
constexpr int kStopChunk = 4;

extern "C" int lrstv_solve(lrstv_handle H, const float* Y, float* X, float* S, int32_t max_iter, double eps,
                           lrstv_report* rep) {
  if (!H || !Y) return fail(LRSTV_ERR_INVALID_ARG, "handle or Y is NULL");
  if (max_iter < 1) return fail(LRSTV_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(eps >= 0.0) && !(eps < 0.0)) return fail(LRSTV_ERR_INVALID_ARG, "eps is NaN");
  int rc = lrstv_reset(H, Y);
  if (rc) return rc;
  const int nc = (int)H->cubes.size();
  const bool test = eps > 0;
  hipStream_t s = H->stream;
  launch_set_double(H->eps, test ? eps : 0.0, s);
  const int chunk = test ? kStopChunk : max_iter;
  int issued = 0, polls = 0;
  bool stop = false;
  while (issued < max_iter && !stop) {
    const int k = (max_iter - issued) < chunk ? (max_iter - issued) : chunk;
    rc = lrstv_iterate(H, k, nullptr);
    if (rc) return rc;
    issued += k;
    if (!test) continue;
    int* buf = H->poll_host + (size_t)(polls & 1) * (nc + 1);
    HIPCHK(hipMemcpyAsync(buf, H->halt, nc * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(buf + nc, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(H->poll_ev[polls & 1], s));
    if (polls > 0) {   // the previous chunk's flags, while this chunk runs
      HIPCHK(hipEventSynchronize(H->poll_ev[(polls - 1) & 1]));
      const int* prev = H->poll_host + (size_t)((polls - 1) & 1) * (nc + 1);
      bool all = true;
      for (int c = 0; c < nc; ++c) all = all && prev[c] != 0;
      stop = all || prev[nc] != 0;
    }
    ++polls;
  }
  std::vector<double> res((size_t)nc * R_COUNT);
  std::vector<int> halted(nc, 0), its(nc, 0);
  int nonfinite = 0;
  HIPCHK(hipMemcpyAsync(res.data(), H->res_last, res.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(halted.data(), H->halt, nc * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(its.data(), H->iters, nc * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&nonfinite, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // later lrstv_iterate calls continue from the stopped state without a test
  launch_set_double(H->eps, 0.0, s);
  launch_fill_int(H->halt, nc, 0, s);
  int status = LRSTV_OK;
  bool bad = nonfinite != 0;
  for (double v : res) bad |= !isfinite(v);
  if (bad) {
    status = fail(LRSTV_ERR_NONFINITE, "non-finite residual within %d iterations", issued);
  } else if (test) {
    bool all = true;
    for (int c = 0; c < nc; ++c) all = all && halted[c] != 0;
    if (!all) {
      status = LRSTV_WARN_NOT_CONVERGED;
      g_err = "stopping test not met within max_iter";
    }
  }
  if (status >= 0) {
    rc = lrstv_read_output(H, X, S);
    if (rc) return rc;
  }
  if (rep) {
    int mx = 0;
    for (int c = 0; c < nc; ++c) mx = its[c] > mx ? its[c] : mx;
    rep->iters = mx;
    for (int r = 0; r < R_COUNT; ++r) {
      double m = 0.0;
      for (int c = 0; c < nc; ++c) m = fmax(m, res[c * R_COUNT + r]);
      rep->residuals[r] = m;
    }
    double mu = 0.0;
    HIPCHK(hipMemcpyAsync(&mu, H->mu, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    rep->mu = mu;
  }
  return status;
}

extern "C" int lrstv_cube_iterations(lrstv_handle H, int32_t* iters, int32_t n) {
  if (!H || !iters) return fail(LRSTV_ERR_INVALID_ARG, "handle or iters is NULL");
  const int nc = (int)H->cubes.size();
  if (n < nc) return fail(LRSTV_ERR_INVALID_ARG, "need room for %d cubes", nc);
  HIPCHK(hipMemcpyAsync(iters, H->iters, nc * sizeof(int), hipMemcpyDeviceToHost, H->stream));
  HIPCHK(hipStreamSynchronize(H->stream));
  return nc;
}

extern "C" int lrstv_get_state(lrstv_handle H, lrstv_state_view* v) {
  if (!H || !v) return fail(LRSTV_ERR_INVALID_ARG, "handle or view is NULL");
  v->X = H->L;
  v->Y = H->O;
  v->Z = H->Z;
  v->S = H->S;
  v->G1 = H->G1;
  v->G2 = H->G2;
  v->F = H->F;
  v->E = H->E;
  v->G3 = H->G3;
  v->G4 = H->G4;
  v->N = H->N;
  v->mu = H->mu;
  v->total = H->total;
  return LRSTV_OK;
}

extern "C" int lrstv_set_state(lrstv_handle H, const lrstv_state_view* v) {
  if (!H || !v) return fail(LRSTV_ERR_INVALID_ARG, "handle or view is NULL");
  if (v->total != H->total) return fail(LRSTV_ERR_INVALID_ARG, "state total %lld != %lld", (long long)v->total,
                                        (long long)H->total);
  if (!v->Z || !v->S || !v->G1 || !v->G2 || !v->F || !v->E || !v->G3 || !v->G4)
    return fail(LRSTV_ERR_INVALID_ARG, "state view lacks a required member");
  const int64_t T = H->total;
  hipStream_t s = H->stream;
  if (v->X) launch_copy(H->L, v->X, T, s);
  if (v->Y) launch_copy(H->O, v->Y, T, s);
  launch_copy(H->Z, v->Z, T, s);
  launch_copy(H->S, v->S, T, s);
  launch_copy(H->G1, v->G1, T, s);
  launch_copy(H->G2, v->G2, T, s);
  launch_copy(H->F, v->F, 3 * T, s);
  launch_copy(H->E, v->E, 3 * T, s);
  launch_copy(H->G3, v->G3, 3 * T, s);
  launch_copy(H->G4, v->G4, 3 * T, s);
  if (v->N) launch_copy(H->N, v->N, T, s);
  if (v->mu) HIPCHK(hipMemcpyAsync(H->mu, v->mu, sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

// ------------------------------------------------------------ adjoint ---
namespace {
struct VjpWs {
  float *dsl, *C, *R, *W, *sig, *ones, *gL, *gZp, *gFp, *dirE, *gA, *gT;
  double *acon, *part;
  int64_t* range;
};
void carve_vjp(const SliceLayout& L, int64_t total, int64_t nmax, int nc, void* base, VjpWs* w, size_t* used) {
  Carve cv(base);
  w->dsl = cv.take<float>(L.slices_floats);
  w->C = cv.take<float>(L.b_floats);
  w->R = cv.take<float>(L.b_floats);
  w->W = cv.take<float>(L.v_floats);
  w->sig = cv.take<float>(L.f_floats);
  w->ones = cv.take<float>(L.f_floats);
  w->acon = cv.take<double>(L.f_floats);
  w->gL = cv.take<float>(total);
  w->gZp = cv.take<float>(total);
  w->gFp = cv.take<float>(3 * total);
  w->dirE = cv.take<float>(3 * total);
  w->gA = cv.take<float>(3 * total);
  w->gT = cv.take<float>(total);
  (void)nmax;
  w->part = cv.take<double>((int64_t)nc * 2 * LRSTV_PARTS);
  w->range = cv.take<int64_t>(2 * (int64_t)nc);
  *used = cv.off + 256;
}
// per cube (or batch element) [first, last) of its slices' columns in the
// fval-shaped arrays
std::vector<int64_t> column_ranges(const SliceLayout& L, int nc) {
  std::vector<int64_t> r(2 * (size_t)nc, 0);
  std::vector<bool> seen(nc, false);
  for (const SliceDesc& d : L.desc) {
    const int64_t a = d.f_off, b = d.f_off + d.n1;
    if (!seen[d.cube]) { r[2 * d.cube] = a; r[2 * d.cube + 1] = b; seen[d.cube] = true; }
    else { if (a < r[2 * d.cube]) r[2 * d.cube] = a; if (b > r[2 * d.cube + 1]) r[2 * d.cube + 1] = b; }
  }
  return r;
}
}  // namespace

extern "C" int lrstv_vjp_workspace_size(lrstv_handle H, size_t* bytes) {
  if (!H || !bytes) return fail(LRSTV_ERR_INVALID_ARG, "handle or bytes is NULL");
  VjpWs w;
  carve_vjp(H->sl, H->total, H->nmax, (int)H->cubes.size(), nullptr, &w, bytes);
  return LRSTV_OK;
}

static bool full_view(const lrstv_state_view* v) {
  return v && v->Z && v->S && v->F && v->E && v->G1 && v->G2 && v->G3 && v->G4;
}

extern "C" int lrstv_iterate_vjp(lrstv_handle H, const lrstv_state_view* before, const lrstv_state_view* after,
                                 const lrstv_state_view* grad_after, const float* grad_X,
                                 lrstv_state_view* grad_before, double* grad_weights, float* grad_Y,
                                 int32_t flags, void* ws, size_t ws_bytes) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  if (H->par.tv != LRSTV_TV_ANISO || H->par.beta > 0 || H->tk_on)
    return fail(LRSTV_ERR_UNSUPPORTED,
                "the adjoint covers the anisotropic full-rank model without the noise term only");
  if (!before || !before->G4 || !before->mu) return fail(LRSTV_ERR_INVALID_ARG, "before needs G4 and mu");
  if (!after || !after->S || !after->F) return fail(LRSTV_ERR_INVALID_ARG, "after needs S and F");
  if (grad_after && !full_view(grad_after))
    return fail(LRSTV_ERR_INVALID_ARG, "grad_after must be NULL or give every state member");
  if (!full_view(grad_before)) return fail(LRSTV_ERR_INVALID_ARG, "grad_before must give every state member");
  if (!grad_weights || !grad_Y || !ws) return fail(LRSTV_ERR_INVALID_ARG, "grad_weights, grad_Y, ws are required");
  const lrstv_state_view* views[4] = {before, after, grad_after, grad_before};
  for (const lrstv_state_view* v : views)
    if (v && v->total != H->total)
      return fail(LRSTV_ERR_INVALID_ARG, "state total %lld != %lld", (long long)v->total, (long long)H->total);
  if (((uintptr_t)ws & 255) != 0) return fail(LRSTV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (flags & ~LRSTV_VJP_INITIAL) return fail(LRSTV_ERR_INVALID_ARG, "unknown flags 0x%x", (unsigned)flags);
  const int nc = (int)H->cubes.size();
  size_t need = 0;
  VjpWs w;
  carve_vjp(H->sl, H->total, H->nmax, nc, nullptr, &w, &need);
  if (ws_bytes < need) return fail(LRSTV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  carve_vjp(H->sl, H->total, H->nmax, nc, ws, &w, &need);
  hipStream_t s = H->stream;
  const double* mu = before->mu;
  const int64_t T = H->total;
  if (H->acon_range.empty()) H->acon_range = column_ranges(H->sl, nc);
  HIPCHK(hipMemcpyAsync(w.range, H->acon_range.data(), H->acon_range.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  launch_fill(w.ones, H->sl.f_floats, 1.f, s);
  auto cube_view = [&](const CubeInfo& ci) {
    VjpCube c;
    const int64_t o = ci.off;
    c.h = ci.h;
    c.w = ci.w;
    c.b = ci.b;
    c.ts = T;
    c.as = T;
    c.G4 = before->G4 + o;
    c.S1 = after->S + o;
    c.F1 = after->F + o;
    const bool ga = grad_after != nullptr;
    c.gaZ = ga ? grad_after->Z + o : nullptr;
    c.gaS = ga ? grad_after->S + o : nullptr;
    c.gaF = ga ? grad_after->F + o : nullptr;
    c.gaE = ga ? grad_after->E + o : nullptr;
    c.gaG1 = ga ? grad_after->G1 + o : nullptr;
    c.gaG2 = ga ? grad_after->G2 + o : nullptr;
    c.gaG3 = ga ? grad_after->G3 + o : nullptr;
    c.gaG4 = ga ? grad_after->G4 + o : nullptr;
    c.gX = grad_X ? grad_X + o : nullptr;
    c.gbZ = grad_before->Z + o;
    c.gbS = grad_before->S + o;
    c.gbF = grad_before->F + o;
    c.gbE = grad_before->E + o;
    c.gbG1 = grad_before->G1 + o;
    c.gbG2 = grad_before->G2 + o;
    c.gbG3 = grad_before->G3 + o;
    c.gbG4 = grad_before->G4 + o;
    c.gL = w.gL + o;
    c.gZp = w.gZp + o;
    c.gFp = w.gFp + o;
    c.dirE = w.dirE + o;
    c.A = H->A + o;
    c.gY = grad_Y + o;
    c.initial = (flags & LRSTV_VJP_INITIAL) != 0;
    return c;
  };
  // 6th and 5th steps; the t-SVT point and direction into Fourier slices
  for (int c = 0; c < nc; ++c) {
    const CubeInfo& ci = H->cubes[c];
    VjpCube vc = cube_view(ci);
    launch_vjp_post(vc, mu, w.part + (int64_t)c * 2 * LRSTV_PARTS + LRSTV_PARTS, s);
    launch_band_dft(H->A + ci.off, T, 3, H->slices + ci.slice_base, ci.h, ci.w, ci.b, s);
    launch_band_dft(w.dirE + ci.off, T, 3, w.dsl + ci.slice_base, ci.h, ci.w, ci.b, s);
  }
  // 4th step: derivative of every slice SVT along its direction
  SvtVjpLaunch J;
  J.fw.desc = H->desc;
  J.fw.n_slices = (int)H->sl.desc.size();
  J.fw.max_n1 = H->sl.max_n1;
  J.fw.min_n1 = H->sl.min_n1;
  J.fw.max_m1 = H->sl.max_m1;
  J.fw.slices = H->slices;
  J.fw.gram = H->gram;
  J.fw.V = H->V;
  J.fw.B = H->B;
  J.fw.tri = H->tri;
  J.fw.xs = H->xs;
  J.fw.Twy = H->Twy;
  J.fw.fval = H->fval;
  J.fw.rcount = H->rcount;
  J.fw.mu = mu;
  J.fw.alpha = H->par.alpha;
  J.fw.thresh = 0.f;
  J.fw.precision = LRSTV_FP32;
  J.fw.tri_variant = H->tri_variant;
  J.dsl = w.dsl;
  J.C = w.C;
  J.R = w.R;
  J.W = w.W;
  J.sig = w.sig;
  J.ones = w.ones;
  J.acon = w.acon;
  launch_svt_vjp(J, s);
  // 3rd, 2nd and 1st steps per cube
  for (int c = 0; c < nc; ++c) {
    const CubeInfo& ci = H->cubes[c];
    VjpCube vc = cube_view(ci);
    float* gA = w.gA + ci.off;
    float2* spec = H->spec + ci.spec_off;
    launch_band_idft(w.dsl + ci.slice_base, 3, gA, T, ci.h, ci.w, ci.b, nullptr, nullptr, nullptr, nullptr, s);
    launch_vjp_shrinkf(vc, gA, mu, w.part + (int64_t)c * 2 * LRSTV_PARTS, s);
    launch_vjp_divt(vc, H->T + ci.off, H->par.w, s);
    launch_rfft_w(H->T + ci.off, spec, ci.h, ci.w, ci.b, s);
    launch_fft_h(spec, ci.h, ci.w, ci.b, -1, s);
    launch_tri_b(spec, ci.h, ci.w, ci.b, H->par.w, mu, 0.0, s);
    launch_fft_h(spec, ci.h, ci.w, ci.b, +1, s);
    launch_irfft_w(spec, w.gT + ci.off, ci.h, ci.w, ci.b, nullptr, s);
    launch_vjp_pre(vc, w.gT + ci.off, H->par.w, mu, s);
  }
  launch_vjp_finish(w.part, w.acon, w.range, nc, grad_weights, s);
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

extern "C" int lrstv_save_state(lrstv_handle H, const lrstv_state_view* dst) {
  if (!H || !full_view(dst)) return fail(LRSTV_ERR_INVALID_ARG, "handle or a destination member is NULL");
  if (dst->total != H->total)
    return fail(LRSTV_ERR_INVALID_ARG, "state total %lld != %lld", (long long)dst->total, (long long)H->total);
  const int64_t T = H->total;
  hipStream_t s = H->stream;
  launch_copy(dst->Z, H->Z, T, s);
  launch_copy(dst->S, H->S, T, s);
  launch_copy(dst->G1, H->G1, T, s);
  launch_copy(dst->G2, H->G2, T, s);
  launch_copy(dst->F, H->F, 3 * T, s);
  launch_copy(dst->E, H->E, 3 * T, s);
  launch_copy(dst->G3, H->G3, 3 * T, s);
  launch_copy(dst->G4, H->G4, 3 * T, s);
  if (dst->N) launch_copy(dst->N, H->N, T, s);
  if (dst->X) launch_copy(dst->X, H->L, T, s);
  if (dst->Y) launch_copy(dst->Y, H->O, T, s);
  if (dst->mu) HIPCHK(hipMemcpyAsync(dst->mu, H->mu, sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

// --------------------------------------------------------- primitives ---

namespace {
struct SvtWs {
  float *slices, *V, *B, *fval, *Twy;
  float2* gram;
  double *tri, *xs;
  int* rcount;
  SliceDesc* desc;
};
void carve_svt(const SliceLayout& L, void* base, SvtWs* w, size_t* used) {
  Carve cv(base);
  w->slices = cv.take<float>(L.slices_floats);
  w->gram = cv.take<float2>(L.gram_c);
  w->V = cv.take<float>(L.v_floats);
  w->B = cv.take<float>(L.b_floats);
  w->tri = cv.take<double>(L.tri_d);
  w->xs = cv.take<double>(L.xs_d);
  w->Twy = cv.take<float>(L.wy_floats);
  w->fval = cv.take<float>(L.f_floats);
  w->rcount = cv.take<int>(L.desc.size());
  w->desc = cv.take<SliceDesc>(L.desc.size());
  *used = cv.off + 256;
}
}  // namespace

__global__ void k_make_desc(SliceDesc* out, int n, int b, int h, int w, int s,
                            int64_t gram_c, int64_t v_f, int64_t b_f, int64_t tri_d, int64_t xs_d, int64_t f_f,
                            int64_t y_f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t hw = (int64_t)h * w;
  const int n1 = h < w ? h : w, m1 = h < w ? w : h;
  SliceDesc d;
  d.h = h;
  d.w = w;
  d.n1 = n1;
  d.m1 = m1;
  d.tall = h >= w;
  d.cube = i / s;
  {
    const int k = i % s;
    d.fw = (float)((k == 0 || 2 * k == b) ? 1 : 2) / (float)b;
  }
  d.a_off = (int64_t)i * 2 * hw;
  d.g_off = (int64_t)i * gram_c;
  d.v_off = (int64_t)i * v_f;
  d.b_off = (int64_t)i * b_f;
  d.t_off = (int64_t)i * tri_d;
  d.x_off = (int64_t)i * xs_d;
  d.f_off = (int64_t)i * f_f;
  d.y_off = (int64_t)i * y_f;
  d.prio = 0;
  d.keep = 0;
  out[i] = d;
}

static SliceLayout svt_layout(int h, int w, int b, int batch) {
  std::vector<CubeInfo> cubes(batch);
  for (int i = 0; i < batch; ++i) {
    cubes[i].h = h;
    cubes[i].w = w;
    cubes[i].b = b;
    cubes[i].s = b / 2 + 1;
    cubes[i].off = 0;
  }
  return make_slices(cubes, 1);
}

extern "C" int lrstv_svt_workspace_size(int32_t h, int32_t w, int32_t b, int32_t batch, int32_t precision,
                                        size_t* bytes) {
  if (!bytes) return fail(LRSTV_ERR_INVALID_ARG, "bytes is NULL");
  int rc = check_dims(h, w, b);
  if (rc) return rc;
  if (batch < 1) return fail(LRSTV_ERR_INVALID_ARG, "batch must be >= 1");
  if (precision != LRSTV_FP32 && precision != LRSTV_SPLIT_BF16)
    return fail(LRSTV_ERR_INVALID_ARG, "unknown precision %d", precision);
  SliceLayout L = svt_layout(h, w, b, batch);
  SvtWs ws;
  carve_svt(L, nullptr, &ws, bytes);
  return LRSTV_OK;
}

extern "C" int lrstv_svt(const float* A, float* E, int32_t h, int32_t w, int32_t b, int32_t batch, float thresh,
                         int32_t precision, void* wsp, size_t ws_bytes, void* stream) {
  size_t need = 0;
  int rc = lrstv_svt_workspace_size(h, w, b, batch, precision, &need);
  if (rc) return rc;
  if (!A || !E || !wsp) return fail(LRSTV_ERR_INVALID_ARG, "A, E and the workspace must be non-NULL");
  if (A == E) return fail(LRSTV_ERR_INVALID_ARG, "E may not alias A");
  if (!(thresh >= 0.f)) return fail(LRSTV_ERR_INVALID_ARG, "thresh must be >= 0");
  if (ws_bytes < need) return fail(LRSTV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (((uintptr_t)wsp & 255) != 0) return fail(LRSTV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  SliceLayout L = svt_layout(h, w, b, batch);
  SvtWs ws;
  carve_svt(L, wsp, &ws, &need);
  const int ns = (int)L.desc.size();
  const int n1 = h < w ? h : w;
  const int64_t hw = (int64_t)h * w;
  prepare_svt(n1);
  hipLaunchKernelGGL(k_make_desc, dim3((ns + 255) / 256), dim3(256), 0, s, ws.desc, ns, (int)b, h, w, b / 2 + 1,
                     (int64_t)n1 * (n1 + 1) / 2, 2 * (int64_t)n1 * n1, 2 * hw, 6 * (int64_t)n1, 3 * (int64_t)n1 * n1,
                     (int64_t)n1, wy_block_floats(n1));
  launch_band_dft(A, (int64_t)b * hw, batch, ws.slices, h, w, b, s);
  SvtLaunch sv;
  sv.desc = ws.desc;
  sv.n_slices = ns;
  sv.max_n1 = L.max_n1;
  sv.min_n1 = L.min_n1;
  sv.max_m1 = L.max_m1;
  sv.slices = ws.slices;
  sv.gram = ws.gram;
  sv.V = ws.V;
  sv.B = ws.B;
  sv.tri = ws.tri;
  sv.xs = ws.xs;
  sv.Twy = ws.Twy;
  sv.fval = ws.fval;
  sv.rcount = ws.rcount;
  sv.mu = nullptr;
  sv.alpha = 0.0;
  sv.thresh = thresh;
  sv.precision = precision;
  launch_svt(sv, s);
  launch_band_idft(ws.slices, batch, E, (int64_t)b * hw, h, w, b, nullptr, nullptr, nullptr, nullptr, s);
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

extern "C" int lrstv_svt_vjp_workspace_size(int32_t h, int32_t w, int32_t b, int32_t batch, size_t* bytes) {
  if (!bytes) return fail(LRSTV_ERR_INVALID_ARG, "bytes is NULL");
  int rc = check_dims(h, w, b);
  if (rc) return rc;
  if (batch < 1) return fail(LRSTV_ERR_INVALID_ARG, "batch must be >= 1");
  SliceLayout L = svt_layout(h, w, b, batch);
  SvtWs sw;
  size_t a = 0, c = 0;
  carve_svt(L, nullptr, &sw, &a);
  VjpWs vw;
  carve_vjp(L, 0, 0, batch, nullptr, &vw, &c);
  *bytes = a + c + 256;
  return LRSTV_OK;
}

extern "C" int lrstv_svt_vjp(const float* A, const float* G, float* gA, int32_t h, int32_t w, int32_t b,
                             int32_t batch, float thresh, double* grad_thresh, void* wsp, size_t ws_bytes,
                             void* stream) {
  size_t need = 0;
  int rc = lrstv_svt_vjp_workspace_size(h, w, b, batch, &need);
  if (rc) return rc;
  if (!A || !G || !gA || !wsp) return fail(LRSTV_ERR_INVALID_ARG, "A, G, gA and the workspace must be non-NULL");
  if (gA == A || gA == G) return fail(LRSTV_ERR_INVALID_ARG, "gA may not alias A or G");
  if (!(thresh >= 0.f)) return fail(LRSTV_ERR_INVALID_ARG, "thresh must be >= 0");
  if (ws_bytes < need) return fail(LRSTV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (((uintptr_t)wsp & 255) != 0) return fail(LRSTV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  SliceLayout L = svt_layout(h, w, b, batch);
  SvtWs sw;
  size_t a = 0, c = 0;
  carve_svt(L, wsp, &sw, &a);
  VjpWs vw;
  void* vbase = (void*)(((uintptr_t)wsp + a + 255) & ~(uintptr_t)255);
  carve_vjp(L, 0, 0, batch, vbase, &vw, &c);
  const int ns = (int)L.desc.size();
  const int n1 = h < w ? h : w;
  const int64_t hw = (int64_t)h * w;
  prepare_svt(n1);
  hipLaunchKernelGGL(k_make_desc, dim3((ns + 255) / 256), dim3(256), 0, s, sw.desc, ns, (int)b, h, w, b / 2 + 1,
                     (int64_t)n1 * (n1 + 1) / 2, 2 * (int64_t)n1 * n1, 2 * hw, 6 * (int64_t)n1, 3 * (int64_t)n1 * n1,
                     (int64_t)n1, wy_block_floats(n1));
  std::vector<int64_t> range = column_ranges(L, batch);
  HIPCHK(hipMemcpyAsync(vw.range, range.data(), range.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  launch_fill(vw.ones, L.f_floats, 1.f, s);
  launch_band_dft(A, (int64_t)b * hw, batch, sw.slices, h, w, b, s);
  launch_band_dft(G, (int64_t)b * hw, batch, vw.dsl, h, w, b, s);
  SvtVjpLaunch J;
  J.fw.desc = sw.desc;
  J.fw.n_slices = ns;
  J.fw.max_n1 = L.max_n1;
  J.fw.min_n1 = L.min_n1;
  J.fw.max_m1 = L.max_m1;
  J.fw.slices = sw.slices;
  J.fw.gram = sw.gram;
  J.fw.V = sw.V;
  J.fw.B = sw.B;
  J.fw.tri = sw.tri;
  J.fw.xs = sw.xs;
  J.fw.Twy = sw.Twy;
  J.fw.fval = sw.fval;
  J.fw.rcount = sw.rcount;
  J.fw.mu = nullptr;
  J.fw.alpha = 0.0;
  J.fw.thresh = thresh;
  J.fw.precision = LRSTV_FP32;
  J.dsl = vw.dsl;
  J.C = vw.C;
  J.R = vw.R;
  J.W = vw.W;
  J.sig = vw.sig;
  J.ones = vw.ones;
  J.acon = vw.acon;
  launch_svt_vjp(J, s);
  launch_band_idft(vw.dsl, batch, gA, (int64_t)b * hw, h, w, b, nullptr, nullptr, nullptr, nullptr, s);
  if (grad_thresh) launch_sum_ranges(vw.acon, vw.range, batch, grad_thresh, s);
  HIPCHK(hipGetLastError());
  // the host range table must outlive the asynchronous copy
  HIPCHK(hipStreamSynchronize(s));
  return LRSTV_OK;
}

extern "C" int lrstv_zsolve_workspace_size(int32_t h, int32_t w, int32_t b, size_t* bytes) {
  if (!bytes) return fail(LRSTV_ERR_INVALID_ARG, "bytes is NULL");
  int rc = check_dims(h, w, b);
  if (rc) return rc;
  *bytes = (size_t)b * h * (w / 2 + 1) * sizeof(float2) + 256;
  return LRSTV_OK;
}

extern "C" int lrstv_zsolve(const float* T, float* Z, int32_t h, int32_t w, int32_t b, double mu, const double wts[3],
                            void* wsp, size_t ws_bytes, void* stream) {
  size_t need = 0;
  int rc = lrstv_zsolve_workspace_size(h, w, b, &need);
  if (rc) return rc;
  if (!T || !Z || !wsp || !wts) return fail(LRSTV_ERR_INVALID_ARG, "NULL pointer argument");
  if (!(mu > 0)) return fail(LRSTV_ERR_INVALID_ARG, "mu must be > 0");
  for (int i = 0; i < 3; ++i)
    if (!(wts[i] >= 0)) return fail(LRSTV_ERR_INVALID_ARG, "weights must be >= 0");
  if (ws_bytes < need) return fail(LRSTV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  float2* spec = (float2*)(((uintptr_t)wsp + 255) & ~(uintptr_t)255);
  launch_rfft_w(T, spec, h, w, b, s);
  launch_fft_h(spec, h, w, b, -1, s);
  launch_tri_b(spec, h, w, b, wts, nullptr, mu, s);
  launch_fft_h(spec, h, w, b, +1, s);
  launch_irfft_w(spec, Z, h, w, b, nullptr, s);
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

// ------------------------------------------- Z-solve without allocation ---
// Scratch of lrstv_zsolve_noalloc: the half spectrum b h (w/2+1) complex of
// one cube, in a file-scope device array (each device holds its own copy,
// loaded with the code object, until the process ends).  Host code never
// passes the array's name to a kernel: it is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress with that device current.
static __device__ __align__(256) float2 scratch[LRSTV_NOALLOC_SCRATCH_BYTES / sizeof(float2)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up on the first
// call per device and kept.
static int scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LRSTV_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LRSTV_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LRSTV_OK;
}

extern "C" int lrstv_zsolve_noalloc(const float* T, float* Z, int32_t h, int32_t w, int32_t b, double mu,
                                    const double wts[3], void* stream) {
  int rc = check_dims(h, w, b);
  if (rc) return rc;
  if (!T || !Z || !wts) return fail(LRSTV_ERR_INVALID_ARG, "NULL pointer argument");
  if (!(mu > 0)) return fail(LRSTV_ERR_INVALID_ARG, "mu must be > 0");
  for (int i = 0; i < 3; ++i)
    if (!(wts[i] >= 0)) return fail(LRSTV_ERR_INVALID_ARG, "weights must be >= 0");
  const size_t need = (size_t)b * h * (w / 2 + 1) * sizeof(float2);
  if (need > LRSTV_NOALLOC_SCRATCH_BYTES)
    return fail(LRSTV_ERR_WORKSPACE, "cube %d x %d x %d needs %zu bytes of scratch, the built-in scratch holds %zu",
                b, h, w, need, (size_t)LRSTV_NOALLOC_SCRATCH_BYTES);
  void* p = nullptr;
  rc = scratch_address(&p);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  float2* spec = (float2*)p;   // every element is written by the forward w transform before it is read
  launch_rfft_w(T, spec, h, w, b, s);
  launch_fft_h(spec, h, w, b, -1, s);
  launch_tri_b(spec, h, w, b, wts, nullptr, mu, s);
  launch_fft_h(spec, h, w, b, +1, s);
  launch_irfft_w(spec, Z, h, w, b, nullptr, s);
  HIPCHK(hipGetLastError());
  return LRSTV_OK;
}

// ----------------------------------------------------------- autotuner ---
static void drop_graph(lrstv_handle_s* H) {
  if (H->gexec) (void)hipGraphExecDestroy(H->gexec);
  if (H->graph) (void)hipGraphDestroy(H->graph);
  H->gexec = nullptr;
  H->graph = nullptr;
}

static SvtLaunch handle_svt(lrstv_handle_s* H) {
  SvtLaunch sv;
  sv.desc = H->desc;
  sv.n_slices = (int)H->sl.desc.size();
  sv.max_n1 = H->sl.max_n1;
  sv.min_n1 = H->sl.min_n1;
  sv.max_m1 = H->sl.max_m1;
  sv.slices = H->slices;
  sv.gram = H->gram;
  sv.V = H->V;
  sv.B = H->B;
  sv.tri = H->tri;
  sv.xs = H->xs;
  sv.Twy = H->Twy;
  sv.fval = H->fval;
  sv.rcount = H->rcount;
  sv.mu = H->mu;
  sv.alpha = H->par.alpha;
  sv.thresh = 0.f;
  sv.precision = H->par.precision;
  sv.tri_variant = H->tri_variant;
  return sv;
}

extern "C" int lrstv_autotune(lrstv_handle H, int32_t reps, lrstv_tuning* out) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  if (reps < 1 || reps > 100) return fail(LRSTV_ERR_INVALID_ARG, "reps must be in [1, 100]");
  hipStream_t s = H->stream;
  SvtLaunch sv = handle_svt(H);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  lrstv_tuning t;
  memset(&t, 0, sizeof t);
  t.n_shapes = kTriVariants;
  int best = -1;
  double best_ms = 0.0;
  hipError_t err = hipSuccess;
  for (int v = 0; v < kTriVariants && err == hipSuccess; ++v) {
    t.shapes_tried[v] = tri_variant_code(v);
    t.tridiag_ms[v] = -1.0;  // not runnable on chip for this batch
    if (!tri_variant_onchip(v, sv.max_n1)) continue;
    sv.tri_variant = v;
    double tot = 0.0;
    for (int r = 0; r <= reps && err == hipSuccess; ++r) {
      // slices of hashed values: full-rank Grams, so no column deflates
      launch_fill_hash(H->slices, H->sl.slices_floats, 0x5eed0000u + (uint32_t)r, s);
      launch_svt_gram(sv, s);
      err = hipEventRecord(e0, s);
      launch_svt_tridiag(sv, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) tot += ms;   // the first run warms up
    }
    t.tridiag_ms[v] = tot / reps;
    if (best < 0 || t.tridiag_ms[v] < best_ms) {
      best = v;
      best_ms = t.tridiag_ms[v];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(LRSTV_ERR_HIP, "autotune: %s", hipGetErrorString(err));
  if (best >= 0 && best != H->tri_variant) {
    H->tri_variant = best;
    drop_graph(H);
  }
  t.tridiag_shape = tri_variant_code(H->tri_variant);
  if (out) *out = t;
  return LRSTV_OK;
}

extern "C" int lrstv_set_tuning(lrstv_handle H, const lrstv_tuning* t) {
  if (!H || !t) return fail(LRSTV_ERR_INVALID_ARG, "handle or tuning is NULL");
  int v = -1;
  for (int i = 0; i < kTriVariants; ++i)
    if (tri_variant_code(i) == t->tridiag_shape) v = i;
  if (v < 0) return fail(LRSTV_ERR_INVALID_ARG, "no tridiagonalisation shape %d", t->tridiag_shape);
  if (v != H->tri_variant) {
    H->tri_variant = v;
    drop_graph(H);
  }
  return LRSTV_OK;
}

extern "C" int lrstv_get_tuning(lrstv_handle H, lrstv_tuning* t) {
  if (!H || !t) return fail(LRSTV_ERR_INVALID_ARG, "handle or tuning is NULL");
  memset(t, 0, sizeof *t);
  t->tridiag_shape = tri_variant_code(H->tri_variant);
  t->n_shapes = kTriVariants;
  for (int v = 0; v < kTriVariants; ++v) {
    t->shapes_tried[v] = tri_variant_code(v);
    t->tridiag_ms[v] = -1.0;
  }
  return LRSTV_OK;
}

// --------------------------------------------------------- diagnostics ---
static const char* kStageNames[ST_COUNT] = {"lrhs", "rfft_w", "fft_h", "tri_b", "irfft_w", "grad_shrink",
                                            "band_dft", "gram", "tridiag", "trieig", "trivec", "backtrans", "bp1",
                                            "colnorm", "bp2", "band_idft", "finish", "hooi"};

extern "C" int lrstv_profile(lrstv_handle H, int32_t enable) {
  if (!H) return fail(LRSTV_ERR_INVALID_ARG, "handle is NULL");
  H->timer.collect(nullptr, nullptr);
  H->timer.on = enable != 0;
  return LRSTV_OK;
}

extern "C" int lrstv_stage_times(lrstv_handle H, double* ms, int32_t* counts, int32_t n) {
  if (!H || !ms || n < LRSTV_NSTAGES) return fail(LRSTV_ERR_INVALID_ARG, "need room for LRSTV_NSTAGES stages");
  int c[ST_COUNT];
  H->timer.collect(ms, c);
  if (counts)
    for (int i = 0; i < ST_COUNT; ++i) counts[i] = c[i];
  return LRSTV_OK;
}

extern "C" int lrstv_slice_ranks(lrstv_handle H, int32_t* ranks, int32_t n) {
  if (!H || !ranks) return fail(LRSTV_ERR_INVALID_ARG, "handle or ranks is NULL");
  const int ns = (int)H->sl.desc.size();
  if (n < ns) return fail(LRSTV_ERR_INVALID_ARG, "need room for %d slices", ns);
  HIPCHK(hipMemcpyAsync(ranks, H->rcount, ns * sizeof(int), hipMemcpyDeviceToHost, H->stream));
  HIPCHK(hipStreamSynchronize(H->stream));
  return ns;
}

extern "C" const char* lrstv_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : "";
}

extern "C" const char* lrstv_status_string(int st) {
  switch (st) {
    case LRSTV_OK: return "ok";
    case LRSTV_WARN_NOT_CONVERGED: return "stopping test not met";
    case LRSTV_ERR_INVALID_ARG: return "invalid argument";
    case LRSTV_ERR_WORKSPACE: return "workspace too small";
    case LRSTV_ERR_UNSUPPORTED: return "unsupported size";
    case LRSTV_ERR_HIP: return "HIP runtime error";
    case LRSTV_ERR_NONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

extern "C" const char* lrstv_last_error(void) { return g_err.c_str(); }

extern "C" int lrstv_version(void) { return 100; }
