// Opt-in per-stage GPU timing: hipEvents recorded around each stage on the
// stream the stage is launched on.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

namespace lrstv {

enum Stage {
  ST_LRHS = 0, ST_RFFT_W, ST_FFT_H, ST_TRI_B, ST_IRFFT_W, ST_GRAD_SHRINK, ST_BAND_DFT, ST_GRAM, ST_TRIDIAG,
  ST_TRIEIG, ST_TRIVEC, ST_BACKTRANS, ST_BP1, ST_COLNORM, ST_BP2, ST_BAND_IDFT, ST_FINISH, ST_HOOI, ST_COUNT
};

struct StageTimer {
  hipStream_t s = nullptr;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ST_COUNT];
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(int st) {
    if (!on) return;
    hipEvent_t a = get();
    if (a) (void)hipEventRecord(a, s);
    ev[st].push_back({a, nullptr});
  }
  void end(int st) {
    if (!on || ev[st].empty()) return;
    hipEvent_t b = get();
    if (b) (void)hipEventRecord(b, s);
    ev[st].back().second = b;
  }
  // Sum of elapsed milliseconds and number of launches per stage; recycles events.
  void collect(double* ms, int* cnt) {
    (void)hipStreamSynchronize(s);
    for (int st = 0; st < ST_COUNT; ++st) {
      double t = 0.0;
      int c = 0;
      for (auto& p : ev[st]) {
        float f = 0.f;
        if (p.first && p.second && hipEventElapsedTime(&f, p.first, p.second) == hipSuccess) {
          t += f;
          ++c;
        }
        if (p.first) pool.push_back(p.first);
        if (p.second) pool.push_back(p.second);
      }
      ev[st].clear();
      if (ms) ms[st] = t;
      if (cnt) cnt[st] = c;
    }
  }
  ~StageTimer() {
    for (int st = 0; st < ST_COUNT; ++st)
      for (auto& p : ev[st]) {
        if (p.first) (void)hipEventDestroy(p.first);
        if (p.second) (void)hipEventDestroy(p.second);
      }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace lrstv
