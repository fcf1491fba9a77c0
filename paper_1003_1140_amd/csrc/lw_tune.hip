// lw_tune.hip -- launch-shape autotuner.
//
// Times candidate launch shapes of one path on a caller-supplied batch with HIP
// events on the context's stream and keeps the fastest:
//   FP32 path: frequencies per thread (1, 2, 4, 8) x particles per work item
//              (automatic, half, double) x plain grid / persistent ticket queue;
//   matrix-core paths: number of frequency bands (1, 2) x contraction tile rows
//              (128, 256).
// The accumulator S is saved before and restored after, so tuning leaves no trace
// in the spectra.  The report (and the optional cache file) is JSON.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <tuple>
#include <vector>

#include "lw_internal.h"
#include "lw_mfma.h"

namespace {

struct Candidate {
  int wpt, pb, persistent, bands, tile;
  double ms;
};

std::string to_json(const Candidate& c) {
  char buf[256];
  snprintf(buf, sizeof(buf),
           "{\"wpt\": %d, \"pb\": %d, \"persistent\": %d, \"bands\": %d, \"tile\": %d, "
           "\"ms\": %.4f}",
           c.wpt, c.pb, c.persistent, c.bands, c.tile, c.ms);
  return buf;
}

}  // namespace

extern "C" lw_status lw_tune(lw_ctx* c, const lw_batch* b, lw_path path, int32_t repeats,
                             const char* cache_json, char* report, size_t report_len) {
  if (!c || !b) return LW_EINVAL;
  if (c->nd <= 0 || c->nw <= 0) {
    c->err = "directions and frequencies must be set before tuning";
    return LW_ESTATE;
  }
  if (b->n_particles <= 0) {
    c->err = "tuning needs a non-empty batch";
    return LW_EINVAL;
  }
  if (repeats < 1) repeats = 1;
  if (path == LW_PATH_AUTO)  // tune the path lw_accumulate would pick
    path = c->nw >= LW_AUTO_MIN_FREQUENCIES ? LW_PATH_MFMA_F16 : LW_PATH_FP32;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != c->device) (void)hipSetDevice(c->device);

  // the accumulator the timed runs add into: S, or the summed amplitudes in coherent synthesis
  double* acc = c->coherent ? c->d_A : c->d_S;
  const size_t nS = (size_t)c->ns * c->nd * c->nw * (c->coherent ? 4 : 1);
  double* saved = nullptr;
  if (hipMalloc(&saved, nS * sizeof(double)) != hipSuccess) {
    c->err = "hipMalloc failed while tuning";
    return LW_ENOMEM;
  }
  (void)hipMemcpyAsync(saved, acc, nS * sizeof(double), hipMemcpyDeviceToDevice, c->stream);

  std::vector<Candidate> cands;
  const bool fp32 = path == LW_PATH_FP32;
  if (fp32) {
    const int auto_wpt = lw::pick_wpt(c->nw);
    const int save_wpt = c->tune_wpt, save_pb = c->tune_pb;
    c->tune_wpt = 0;
    c->tune_pb = 0;
    const int auto_pb = lw::direct_shape(c, b->n_particles).pb;
    c->tune_wpt = save_wpt;
    c->tune_pb = save_pb;
    for (int wpt : {1, 2, 4, 8}) {
      if (wpt > 2 * auto_wpt) continue;
      for (int pb : {auto_pb, std::max(1, auto_pb / 2), std::min(4096, auto_pb * 2)})
        for (int pers : {0, 1}) cands.push_back({wpt, pb, pers, 0, 0, 0.0});
    }
    std::sort(cands.begin(), cands.end(), [](const Candidate& x, const Candidate& y) {
      return std::make_tuple(x.wpt, x.pb, x.persistent) < std::make_tuple(y.wpt, y.pb, y.persistent);
    });
    cands.erase(std::unique(cands.begin(), cands.end(),
                            [](const Candidate& x, const Candidate& y) {
                              return x.wpt == y.wpt && x.pb == y.pb && x.persistent == y.persistent;
                            }),
                cands.end());
  } else {
    for (int bands : {1, 2})
      for (int tile : {1, 2, 3, 4}) cands.push_back({0, 0, 1, bands, tile, 0.0});
  }

  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  lw_status st = LW_OK;
  const bool prof = c->prof;
  c->prof = false;
  for (Candidate& cd : cands) {
    cd.ms = -1.0;
    if (fp32)
      st = lw_set_tuning(c, cd.wpt, cd.pb, cd.persistent, 0, 0);
    else
      st = lw_set_tuning(c, c->tune_wpt, c->tune_pb, c->tune_persistent, cd.bands, cd.tile);
    if (st != LW_OK) break;
    if (fp32 && cd.persistent) {
      st = lw_plan_batch(c, b, path);
      if (st != LW_OK) break;
    }
    size_t bytes = 0;
    st = lw_workspace_size(c, b, path, &bytes);
    if (st != LW_OK) break;
    void* ws = nullptr;
    if (bytes > 0 && hipMalloc(&ws, bytes) != hipSuccess) {
      c->err = "hipMalloc failed while tuning";
      st = LW_ENOMEM;
      break;
    }
    st = lw_accumulate(c, b, path, ws, bytes, nullptr);  // warm-up
    if (st == LW_OK) {
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < repeats && st == LW_OK; ++r) st = lw_accumulate(c, b, path, ws, bytes, nullptr);
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      cd.ms = ms / repeats;
    }
    (void)hipStreamSynchronize(c->stream);
    if (ws) (void)hipFree(ws);
    if (st != LW_OK) break;
  }
  c->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the accumulator
  (void)hipMemcpyAsync(acc, saved, nS * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(saved);
  if (st != LW_OK) {
    if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
    return st;
  }
  const Candidate* best = nullptr;
  for (const Candidate& cd : cands)
    if (cd.ms >= 0.0 && (!best || cd.ms < best->ms)) best = &cd;
  if (best) {
    if (fp32) {
      st = lw_set_tuning(c, best->wpt, best->pb, best->persistent, 0, 0);
      if (st == LW_OK && best->persistent) st = lw_plan_batch(c, b, path);
    } else {
      st = lw_set_tuning(c, c->tune_wpt, c->tune_pb, c->tune_persistent, best->bands, best->tile);
    }
  }
  std::string js = std::string("{\"path\": ") + std::to_string((int)path) + ", \"best\": " +
                   (best ? to_json(*best) : std::string("null")) + ", \"candidates\": [";
  for (size_t i = 0; i < cands.size(); ++i) js += (i ? ", " : "") + to_json(cands[i]);
  js += "]}";
  if (report && report_len > 0) {
    strncpy(report, js.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  if (cache_json && cache_json[0]) {
    FILE* f = fopen(cache_json, "w");
    if (f) {
      fputs(js.c_str(), f);
      fputc('\n', f);
      fclose(f);
    } else if (st == LW_OK) {
      c->err = std::string("cannot write ") + cache_json;
      st = LW_EINVAL;
    }
  }
  if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
  return st;
}
