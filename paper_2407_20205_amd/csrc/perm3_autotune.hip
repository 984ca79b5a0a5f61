// perm_autotune / perm_autotune_batch: pick the block decomposition of the
// Gray range (Section 3.1) for one class of calls by timing it on the device.
//
// The decomposition never changes a result, only how the 2^n Gray indices are
// shared out: the persistent waves per SIMD, the per-lane chunk length (its
// cap chunk_log_max, the tasks each wave should get, and the bounds on the
// tasks of one matrix), body_log (the shortest chunk), the chunks a lane
// walks per task and, for small n, the order at or below which every index is
// tested exactly.  Candidates differ from the class's current tuning in those
// fields only.  The search is successive halving (Jamieson and Talwalkar,
// "Non-stochastic best arm identification and hyperparameter optimization",
// 2016): every candidate is timed once, the faster half is timed again with
// twice the repetitions, and so on until one is left or the time budget is
// spent; the class's current tuning is always among the candidates, so the
// winner is never slower than it on the tuner's own measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_runtime.h"

using namespace perm3;

namespace {

// splitmix64: a fixed, published generator for the synthetic entries
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Set the body_log (chunks of at least 2^(body_log+1) indices, the fast walk
// from n = body_log + 7) that applies to matrices of order n.
void set_block(perm_tuning &t, int n, int bl)
{
    if (n <= t.mid_max_n) t.body_log_mid = bl; else t.body_log = bl;
    if (t.direct_max_n < t.body_log_mid + 6) t.direct_max_n = t.body_log_mid + 6;
    if (t.direct_max_n < t.body_log + 6) t.direct_max_n = t.body_log + 6;
}

bool same_tuning(const perm_tuning &a, const perm_tuning &b) { return memcmp(&a, &b, sizeof a) == 0; }

void add_unique(std::vector<perm_tuning> &v, const perm_tuning &t)
{
    if (!tuning_valid(t)) return;
    for (const perm_tuning &u : v)
        if (same_tuning(u, t)) return;
    v.push_back(t);
}

// Candidates for one matrix of order n, by class, around the current tuning.
std::vector<perm_tuning> single_candidates(const perm_tuning &base, int cls, int n)
{
    std::vector<perm_tuning> v;
    v.push_back(base);
    if (cls == PERM_TUNE_LARGE) {
        for (int wp : {8, 6, 4})
            for (int bl : {5, 6})
                for (int st : {1, 2})
                    for (int tpw : {16, 8, 32})
                        for (int cl : {20, 18, 22}) {
                            perm_tuning t = base;
                            t.waves_per_simd = wp;
                            t.states_per_lane = st;
                            t.tasks_per_wave = tpw;
                            t.chunk_log_max = cl;
                            set_block(t, n, bl);
                            add_unique(v, t);
                        }
    } else if (cls == PERM_TUNE_MID) {
        for (int wp : {8, 4})
            for (int bl : {4, 5})
                for (int mt : {10, 8, 6})
                    for (int ml : {19, 17, 21})
                        for (int cl : {20, 16}) {
                            perm_tuning t = base;
                            t.waves_per_simd = wp;
                            t.max_tasks_log = mt;
                            t.min_task_log = ml;
                            t.chunk_log_max = cl;
                            set_block(t, n, bl);
                            add_unique(v, t);
                        }
    } else {
        for (int wp : {8, 4})
            for (int dm : {11, 14, 17})
                for (int mt : {10, 8, 6, 4})
                    for (int bl : {4, 5}) {
                        perm_tuning t = base;
                        t.waves_per_simd = wp;
                        t.max_tasks_log = mt;
                        t.direct_max_n = dm;
                        set_block(t, n, bl);
                        add_unique(v, t);
                    }
    }
    return v;
}

// Candidates for a batch of mixed orders.
std::vector<perm_tuning> batch_candidates(const perm_tuning &base)
{
    std::vector<perm_tuning> v;
    v.push_back(base);
    for (int wp : {8, 6})
        for (int blm : {4, 5})
            for (int mid : {31, 26, 23})
                for (int tpw : {16, 8, 32})
                    for (int st : {1, 2})
                        for (int cl : {20, 18}) {
                            perm_tuning t = base;
                            t.waves_per_simd = wp;
                            t.body_log_mid = blm;
                            t.mid_max_n = mid;
                            t.tasks_per_wave = tpw;
                            t.states_per_lane = st;
                            t.chunk_log_max = cl;
                            if (t.direct_max_n < blm + 6) t.direct_max_n = blm + 6;
                            add_unique(v, t);
                        }
    return v;
}

// Successive halving over `cands`; time(t, reps) returns the mean time of
// reps runs with tuning t installed (negative on error, with rc set).
template <typename TimeFn>
int32_t halve(Context *c, int cls, std::vector<perm_tuning> cands, int32_t budget_ms, TimeFn time,
              perm_tuning *best)
{
    const perm_tuning saved = c->tunings[cls];
    const int32_t saved_src = c->tune_src[cls];
    const auto t0 = Clock::now();
    int reps = 1;
    std::vector<std::pair<double, perm_tuning>> scored;
    for (bool first = true; cands.size() > 1; first = false) {
        if (!first && ms_since(t0) > budget_ms) break;
        scored.clear();
        for (const perm_tuning &t : cands) {
            c->set_tuning(cls, t, saved_src);
            double ms = 0.0;
            const int32_t rc = time(reps, &ms);
            if (rc) {
                c->set_tuning(cls, saved, saved_src);
                return rc;
            }
            scored.emplace_back(ms, t);
        }
        std::stable_sort(scored.begin(), scored.end(),
                         [](const std::pair<double, perm_tuning> &a, const std::pair<double, perm_tuning> &b) {
                             return a.first < b.first;
                         });
        cands.clear();
        for (size_t k = 0; k < (scored.size() + 1) / 2; ++k) cands.push_back(scored[k].second);
        reps *= 2;
    }
    c->set_tuning(cls, cands.front(), PERM_TUNE_SRC_AUTOTUNE);
    *best = cands.front();
    return PERM_OK;
}

}  // namespace

extern "C" int32_t perm_autotune(int32_t n, int32_t budget_ms, perm_tuning *best)
{
    if (!best) return set_error(PERM_EINVAL, "null pointer");
    if (n < 12 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "autotune needs 12 <= n <= 63");
    if (budget_ms < 1) budget_ms = 1;
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;

    std::vector<uint8_t> A((size_t)n * n);
    uint64_t s = 0x5EED0000ull + (uint64_t)n;
    for (auto &x : A) x = (uint8_t)(splitmix64(s) % 3);
    const uint8_t *As[1] = {A.data()};
    int32_t ns[1] = {n};
    const int cls = tune_class_host(1, n);
    // the large class: the walk kernel over up to 2^36 indices, by its HIP events
    const int span_log = n < 36 ? n : 36;
    const uint64_t hi = 1ull << span_log;

    std::lock_guard<std::mutex> g(c->mu);
    const bool timing_was = timing_enabled();
    perm_timing_enable(cls == PERM_TUNE_LARGE ? 1 : 0);
    auto time = [&](int reps, double *ms) -> int32_t {
        int64_t tally = 0;
        uint8_t r = 0;
        // one untimed call: first use of a shape
        int32_t e = cls == PERM_TUNE_LARGE ? c->run_host(As, ns, 1, true, 0, hi, nullptr, &tally)
                                           : c->run_host(As, ns, 1, false, 0, 0, &r, nullptr);
        if (e) return e;
        double sum = 0.0;
        for (int k = 0; k < reps; ++k) {
            if (cls == PERM_TUNE_LARGE) {
                if ((e = c->run_host(As, ns, 1, true, 0, hi, nullptr, &tally))) return e;
                perm_timing tm;
                if ((e = c->timing(&tm))) return e;
                sum += tm.hot_kernel_ms;
            } else {
                const auto a = Clock::now();
                if ((e = c->run_host(As, ns, 1, false, 0, 0, &r, nullptr))) return e;
                sum += ms_since(a);
            }
        }
        *ms = sum / reps;
        return PERM_OK;
    };
    // the short calls of the small classes are timed over more repetitions
    const int scale = cls == PERM_TUNE_LARGE ? 1 : 16;
    rc = halve(c, cls, single_candidates(c->tunings[cls], cls, n), budget_ms,
               [&](int reps, double *ms) { return time(reps * scale, ms); }, best);
    perm_timing_enable(timing_was ? 1 : 0);
    return rc;
}

extern "C" int32_t perm_autotune_batch(const uint64_t *planes_dev, const int64_t *row_off_dev, const int32_t *ns_dev,
                                       int32_t count, uint8_t *out_dev, int32_t budget_ms, perm_tuning *best)
{
    if (!best) return set_error(PERM_EINVAL, "null pointer");
    if (count < 2 || count > PERM_MAX_BATCH) return set_error(PERM_EINVAL, "count = %d out of range", count);
    if (!planes_dev || !row_off_dev || !ns_dev || !out_dev) return set_error(PERM_EINVAL, "null pointer argument");
    if (budget_ms < 1) budget_ms = 1;
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    if ((rc = c->reserve_work(count, (int64_t)count * PERM_MAX_N))) return rc;
    Launch L;
    memset(&L, 0, sizeof L);
    L.pack_kind = 1;
    L.planes_dev = planes_dev;
    L.row_off_dev = row_off_dev;
    L.ns_dev = ns_dev;
    L.count = count;
    L.out_dev = out_dev;
    L.cls = PERM_TUNE_BATCH;
    L.defer = 1;
    const bool timing_was = timing_enabled();
    perm_timing_enable(1);
    // timed calls run eagerly on the library stream (no graph), all launches between two events
    auto time = [&](int reps, double *ms) -> int32_t {
        double sum = 0.0;
        for (int k = 0; k < reps; ++k) {
            int32_t e = c->run(L, c->stream, false);
            if (e) return e;
            perm_timing tm;
            if ((e = c->timing(&tm))) return e;
            sum += tm.total_ms;
        }
        *ms = sum / reps;
        return PERM_OK;
    };
    rc = halve(c, PERM_TUNE_BATCH, batch_candidates(c->tunings[PERM_TUNE_BATCH]), budget_ms, time, best);
    perm_timing_enable(timing_was ? 1 : 0);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return PERM_OK;
}
