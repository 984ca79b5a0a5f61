// perm_autotune: pick the walk's launch shape by timing it on the device.
//
// Candidates vary the persistent waves per SIMD, the chunks each lane walks
// side by side, the unrolled block length (2^body_log Gray steps), the task
// granularity and, for small n, the size at or below which every index is
// tested exactly.  Each candidate walks the
// same pseudo-random matrix of the requested n over a Gray index range long
// enough to fill the machine; the one with the most indices per second wins
// and becomes the context's tuning.
#include <hip/hip_runtime.h>

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

    // range long enough to keep every candidate's machine busy for a few ms
    const int span_log = n < 34 ? n : 34;
    const uint64_t hi = 1ull << span_log;

    std::lock_guard<std::mutex> g(c->mu);
    const perm_tuning saved = c->tuning;
    perm_tuning top = saved;
    double top_rate = -1.0;
    const auto t0 = std::chrono::steady_clock::now();
    const int wps[] = {4, 8, 12, 16, 2};
    const int bls[] = {5, 6, 4};
    const int tpws[] = {8, 4, 16};
    const int dmx[] = {16, 20, 14, 24};
    const int ndm = n <= 24 ? 4 : 1;
    const int sts[] = {2, 1, 4};

    for (int di = 0; di < ndm; ++di)
      for (int st : sts)
        for (int bl : bls)
            for (int tpw : tpws)
                for (int wp : wps) {
                    const double spent = std::chrono::duration<double, std::milli>(
                                             std::chrono::steady_clock::now() - t0).count();
                    if (spent > budget_ms && top_rate > 0) goto done;
                    perm_tuning t = saved;
                    t.waves_per_simd = wp;
                    t.body_log = bl;
                    t.tasks_per_wave = tpw;
                    t.direct_max_n = dmx[di] < bl + 6 ? bl + 6 : dmx[di];
                    t.states_per_lane = st;
                    // the candidate block length applies to matrices of this n
                    if (n <= t.mid_max_n) t.body_log_mid = bl; else t.body_log = bl;
                    if (t.direct_max_n < t.body_log_mid + 6) t.direct_max_n = t.body_log_mid + 6;
                    if (!tuning_valid(t)) continue;
                    c->tuning = t;
                    const uint8_t *As[1] = {A.data()};
                    int32_t ns[1] = {n};
                    int64_t tally = 0;
                    // warm once, then time
                    rc = c->run_host(As, ns, 1, true, 0, hi, nullptr, &tally);
                    if (rc) goto fail;
                    const auto a = std::chrono::steady_clock::now();
                    rc = c->run_host(As, ns, 1, true, 0, hi, nullptr, &tally);
                    if (rc) goto fail;
                    const double sec =
                        std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
                    const double rate = (double)hi / (sec > 0 ? sec : 1e-9);
                    if (rate > top_rate) {
                        top_rate = rate;
                        top = t;
                    }
                }
done:
    c->tuning = top;
    c->drop_graphs();
    *best = top;
    return PERM_OK;
fail:
    c->tuning = saved;
    return rc;
}
