// api_common.hip -- error reporting, problem validation and the size query of
// the C ABI.
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace dst {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ------------------------------------------------------------ kernel timers
namespace {
struct TimedLaunch {
  int kind;
  hipEvent_t ev[2];
};
std::mutex g_kt_mu;
bool g_kt_on = false;
std::vector<TimedLaunch> g_kt;   // launches recorded since timing was switched on
std::vector<hipEvent_t> g_kt_pool;

hipEvent_t kt_event() {
  if (!g_kt_pool.empty()) {
    hipEvent_t e = g_kt_pool.back();
    g_kt_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void kt_clear() {
  for (TimedLaunch &t : g_kt) {
    g_kt_pool.push_back(t.ev[0]);
    g_kt_pool.push_back(t.ev[1]);
  }
  g_kt.clear();
}
}  // namespace

int kt_start(int kind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_kt_mu);
  if (!g_kt_on) return -1;
  TimedLaunch t{kind, {kt_event(), kt_event()}};
  if (!t.ev[0] || !t.ev[1] || hipEventRecord(t.ev[0], s) != hipSuccess) return -1;
  g_kt.push_back(t);
  return (int)g_kt.size() - 1;
}

void kt_stop(int token, hipStream_t s) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_kt_mu);
  if (token < (int)g_kt.size()) (void)hipEventRecord(g_kt[token].ev[1], s);
}

int validate_problem(const dirac_st_problem *p) {
  DST_CHECK(p != nullptr, "problem is NULL");
  DST_CHECK(p->d >= 1 && p->d <= 3, "d must be 1, 2 or 3 (got %d)", p->d);
  DST_CHECK(p->nc == (p->d == 3 ? 4 : 2), "nc must be %d for d = %d (got %d)", p->d == 3 ? 4 : 2,
            p->d, p->nc);
  DST_CHECK(p->n[0] >= 1, "n[0] (time elements) must be >= 1");
  for (int a = 1; a <= p->d; a++)
    DST_CHECK(p->n[a] >= 3, "n[%d] must be >= 3 on the periodic axis (got %d)", a, p->n[a]);
  for (int a = 0; a <= p->d; a++)
    DST_CHECK(p->len[a] > 0.0, "len[%d] must be positive", a);
  DST_CHECK(p->vkind >= 0 && p->vkind <= 2, "unknown potential kind %d", p->vkind);
  DST_CHECK(p->vkind != 2 || p->lw > 0.0, "smooth step needs lw > 0");
  int64_t S = spatial_nodes(p);
  DST_CHECK(total_blocks(p) < (int64_t)INT32_MAX && S * p->n[0] < (int64_t)INT32_MAX,
            "problem too large for int32 block indices");
  return 0;
}

int64_t spatial_nodes(const dirac_st_problem *p) {
  int64_t s = 1;
  for (int a = 1; a <= p->d; a++) s *= p->n[a];
  return s;
}

int blocks_per_row(const dirac_st_problem *p, int tau) {
  int ct = 1 + (tau >= 2) + (tau <= p->n[0] - 1);
  int s = 1;
  for (int a = 0; a < p->d; a++) s *= 3;
  return ct * s;
}

int64_t total_blocks(const dirac_st_problem *p) {
  int64_t S = spatial_nodes(p), tot = 0;
  const int nt = p->n[0];
  if (nt == 1) return S * blocks_per_row(p, 1);
  tot += S * blocks_per_row(p, 1);
  tot += S * blocks_per_row(p, nt);
  if (nt > 2) tot += (int64_t)(nt - 2) * S * blocks_per_row(p, 2);
  return tot;
}

}  // namespace dst

extern "C" const char *dirac_st_last_error(void) { return dst::g_err; }

extern "C" int dirac_st_sizes(const dirac_st_problem *prob, int64_t *nrows, int64_t *nnzb) {
  dst::clear_error();
  if (int rc = dst::validate_problem(prob)) return rc;
  DST_CHECK(nrows && nnzb, "null output pointer");
  *nrows = dst::spatial_nodes(prob) * prob->n[0];
  *nnzb = dst::total_blocks(prob);
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_timing(int32_t on) {
  dst::clear_error();
  std::lock_guard<std::mutex> lk(dst::g_kt_mu);
  dst::kt_clear();
  dst::g_kt_on = on != 0;
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_timing_read(int32_t kind, int64_t *count, double *total_ms) {
  dst::clear_error();
  DST_CHECK(count && total_ms, "count and total_ms must be set");
  DST_CHECK(kind >= 0 && kind < DIRAC_ST_TIMED_COUNT, "unknown timed kernel %d", kind);
  std::lock_guard<std::mutex> lk(dst::g_kt_mu);
  int64_t n = 0;
  double ms = 0.0;
  for (const auto &t : dst::g_kt) {
    if (t.kind != kind) continue;
    DST_HIP(hipEventSynchronize(t.ev[1]));
    float e = 0.f;
    DST_HIP(hipEventElapsedTime(&e, t.ev[0], t.ev[1]));
    ms += e;
    n++;
  }
  *count = n;
  *total_ms = ms;
  return DIRAC_ST_OK;
}
