// Per-kernel timing for measurement harnesses.  Off by default; when on,
// each library launch is bracketed by a pair of HIP events recorded on the
// launch's own stream, and filed under its operation tag together with the
// algorithmic bytes and flops of that launch.  Collection waits for the
// recorded events and aggregates per tag.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace dlm {
namespace {

struct Pending {
  std::string tag;
  hipEvent_t a = nullptr, b = nullptr;
  double bytes = 0, flops = 0;
};

struct Agg {
  std::string tag;
  double ms = 0, bytes = 0, flops = 0;
  int64_t n = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_aggs;
thread_local Pending t_cur;
thread_local bool t_open = false;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void collect_locked() {
  for (Pending &p : g_pending) {
    float ms = 0.f;
    if (p.a && p.b && hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      Agg *dst = nullptr;
      for (Agg &g : g_aggs)
        if (g.tag == p.tag) dst = &g;
      if (!dst) {
        g_aggs.push_back(Agg{p.tag});
        dst = &g_aggs.back();
      }
      dst->ms += ms;
      dst->bytes += p.bytes;
      dst->flops += p.flops;
      dst->n += 1;
    }
    if (p.a) g_pool.push_back(p.a);
    if (p.b) g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace

bool timing_on() { return g_on; }

void timing_begin(const char *tag, void *stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  t_cur = Pending{};
  t_cur.tag = tag;
  t_cur.a = take_event();
  t_cur.b = take_event();
  if (t_cur.a) (void)hipEventRecord(t_cur.a, (hipStream_t)stream);
  t_open = true;
}

void timing_end(void *stream, double alg_bytes, double alg_flops) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!t_open) return;
  if (t_cur.b) (void)hipEventRecord(t_cur.b, (hipStream_t)stream);
  t_cur.bytes = alg_bytes;
  t_cur.flops = alg_flops;
  g_pending.push_back(t_cur);
  t_open = false;
}

}  // namespace dlm

using namespace dlm;

extern "C" {

dlm_status dlm_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return DLM_OK;
}

dlm_status dlm_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  collect_locked();
  g_aggs.clear();
  return DLM_OK;
}

int dlm_timing_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  collect_locked();
  return int(g_aggs.size());
}

dlm_status dlm_timing_entry(int i, char *tag, size_t tag_len, double *total_ms, int64_t *launches,
                            double *alg_bytes, double *alg_flops) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (i < 0 || i >= int(g_aggs.size())) return DLM_EINVAL;
  const Agg &a = g_aggs[i];
  if (tag && tag_len > 0) {
    const size_t n = a.tag.size() < tag_len - 1 ? a.tag.size() : tag_len - 1;
    a.tag.copy(tag, n);
    tag[n] = '\0';
  }
  if (total_ms) *total_ms = a.ms;
  if (launches) *launches = a.n;
  if (alg_bytes) *alg_bytes = a.bytes;
  if (alg_flops) *alg_flops = a.flops;
  return DLM_OK;
}

}  // extern "C"
