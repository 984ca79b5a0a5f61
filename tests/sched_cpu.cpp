// The serving scheduler (paper_2407_20205_amd/csrc/perm3_sched.hpp) on the
// CPU, built under ThreadSanitizer, with a mock executor in place of the GPU.
//
// The mock's "device" is a thread: a launched tick's tasks are walked there
// by the CPU oracle (oracle/perm3_oracle.c, T over each task's Gray range,
// Sections 3 and 3.1), added to the slot's tally, and a finishing slot's
// result is (-1)^n T mod 3 (eq. (2)).  The fast lane asks the oracle for
// perm mod 3 directly.  The mock also checks the scheduler's contract: each
// slot's Gray range is covered once, in order, by its tasks; no tick is
// launched while another is in flight; admission respects the slots and the
// work budget.  Faults can be injected: a failed launch, a failed fast-lane
// call, or a tick that never finishes (for the watchdog).
//
//   sched_cpu <seed> <count> <policy> <max_slots> <budget_log> <quantum_log> <fast_n>
//             <submitters> <queue_cap> <fault> <fault_at> <n_lo> <n_hi> <timeout_ms>
//
// fault: none | launch | fast | hang.  budget_log 0 = no budget.  Prints
// "ok ..." and exits 0 when every check passes.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "perm3_sched.hpp"

extern "C" {
int64_t oracle_range_tally(const uint8_t *A, int n, uint64_t a, uint64_t b, int *ok);
int oracle_perm_mod3(const uint8_t *A, int n, int nthreads);
}

using namespace perm3;

static std::atomic<int> g_errors{0};

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                        \
            g_errors++;                                   \
        }                                                 \
    } while (0)

struct MockSlot {
    bool active = false;
    int n = 0;
    std::vector<uint8_t> A;
    int64_t tally = 0;
    uint64_t next_index = 0;   // the first Gray index no task has covered yet
};

struct MockExecutor final : SchedExecutor {
    enum Fault { NONE, LAUNCH, FAST, HANG };
    Fault fault = NONE;
    int fault_at = -1;
    uint64_t budget = 0;
    int max_slots = 0;

    std::vector<MockSlot> slots;
    uint64_t active_work = 0;
    int launches = 0, fast_calls = 0;
    bool in_flight = false;

    // the device thread and its one tick at a time
    std::mutex mu;
    std::condition_variable cv;
    bool have_job = false, job_done = false, quit = false, released = false, hang_this = false;
    std::vector<TickTask> job_tasks;
    std::vector<int32_t> job_fin;
    std::vector<uint8_t> job_out;
    std::atomic<bool> done_flag{false};
    std::thread dev;

    explicit MockExecutor(int slots_) : max_slots(slots_)
    {
        slots.resize((size_t)slots_);
        dev = std::thread([this] { device(); });
    }
    ~MockExecutor() override
    {
        {
            std::lock_guard<std::mutex> g(mu);
            quit = true;
            released = true;
        }
        cv.notify_all();
        dev.join();
    }

    void device()
    {
        std::unique_lock<std::mutex> g(mu);
        for (;;) {
            cv.wait(g, [&] { return quit || have_job; });
            if (!have_job) return;
            if (hang_this) {
                // a tick that never ends: held until the executor is torn down
                cv.wait(g, [&] { return released; });
                have_job = false;
                return;
            }
            std::vector<TickTask> tasks = job_tasks;
            std::vector<int32_t> fin = job_fin;
            g.unlock();
            for (const TickTask &t : tasks) {
                MockSlot &sl = slots[t.slot];
                const uint64_t total = 1ull << sl.n;
                const uint64_t a = t.c_first << t.m;
                uint64_t b = (t.c_first + (uint64_t)t.nchunks) << t.m;
                if (b > total) b = total;
                CHECK(sl.active, "task of slot %d, which holds no request", t.slot);
                CHECK(a == sl.next_index, "slot %d: task starts at %llu, expected %llu", t.slot,
                      (unsigned long long)a, (unsigned long long)sl.next_index);
                CHECK(t.nchunks >= 1 && t.nchunks <= 64, "task of %d chunks", t.nchunks);
                int ok = 0;
                sl.tally += oracle_range_tally(sl.A.data(), sl.n, a, b, &ok);
                CHECK(ok, "oracle refused [%llu, %llu) of n = %d", (unsigned long long)a, (unsigned long long)b,
                      sl.n);
                sl.next_index = b;
            }
            std::vector<uint8_t> out(fin.size());
            for (size_t i = 0; i < fin.size(); ++i) {
                MockSlot &sl = slots[fin[i]];
                CHECK(sl.next_index == (1ull << sl.n), "slot %d finishes at %llu of 2^%d", fin[i],
                      (unsigned long long)sl.next_index, sl.n);
                const int64_t p = (sl.n & 1) ? -sl.tally : sl.tally;   // eq. (2): (-1)^n T
                out[i] = (uint8_t)(((p % 3) + 3) % 3);
            }
            g.lock();
            job_out = out;
            have_job = false;
            job_done = true;
            done_flag.store(true);
            cv.notify_all();
        }
    }

    int32_t admit(int s, const Request &r) override
    {
        CHECK(s >= 0 && s < max_slots, "slot %d out of range", s);
        MockSlot &sl = slots[s];
        CHECK(!sl.active, "slot %d admitted twice", s);
        const uint64_t work = 1ull << r.n;
        CHECK(budget == 0 || active_work == 0 || active_work + work <= budget,
              "admission past the budget: %llu + %llu > %llu", (unsigned long long)active_work,
              (unsigned long long)work, (unsigned long long)budget);
        sl.active = true;
        sl.n = r.n;
        sl.A = r.A;
        sl.tally = 0;
        sl.next_index = 0;
        active_work += work;
        return PERM_OK;
    }

    int32_t launch(const TickTask *tasks, size_t nt, const int32_t *fin, uint32_t nfin) override
    {
        CHECK(!in_flight, "a tick launched while another is in flight");
        const int k = launches++;
        if (fault == LAUNCH && k == fault_at) return PERM_EDEVICE;
        std::lock_guard<std::mutex> g(mu);
        job_tasks.assign(tasks, tasks + nt);
        job_fin.assign(fin, fin + nfin);
        have_job = true;
        job_done = false;
        hang_this = fault == HANG && k == fault_at;
        done_flag.store(false);
        in_flight = true;
        cv.notify_all();
        return PERM_OK;
    }

    int32_t query(bool *finished) override
    {
        *finished = done_flag.load();
        return PERM_OK;
    }

    int32_t complete(uint8_t *fin_out) override
    {
        std::unique_lock<std::mutex> g(mu);
        cv.wait(g, [&] { return job_done; });
        for (size_t i = 0; i < job_fin.size(); ++i) {
            fin_out[i] = job_out[i];
            MockSlot &sl = slots[job_fin[i]];
            active_work -= 1ull << sl.n;
            sl.active = false;
        }
        in_flight = false;
        return PERM_OK;
    }

    int32_t run_fast(const uint8_t *const *As, const int32_t *ns, int32_t count, uint8_t *out) override
    {
        const int k = fast_calls++;
        if (fault == FAST && k == fault_at) return PERM_EDEVICE;
        CHECK(count >= 1 && count <= SMALL_PLAN_MAX, "fast batch of %d", count);
        uint64_t work = 0;
        for (int32_t i = 0; i < count; ++i) {
            out[i] = (uint8_t)oracle_perm_mod3(As[i], ns[i], 1);
            work += 1ull << ns[i];
        }
        CHECK(count == 1 || work <= SMALL_FUSED_WORK, "fast batch of %llu indices", (unsigned long long)work);
        return PERM_OK;
    }
};

static uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(int argc, char **argv)
{
    if (argc != 15) {
        fprintf(stderr, "usage: see the header comment\n");
        return 2;
    }
    uint64_t seed = strtoull(argv[1], nullptr, 10);
    const int count = atoi(argv[2]);
    const int policy = atoi(argv[3]);
    const int max_slots = atoi(argv[4]);
    const int budget_log = atoi(argv[5]);
    const int quantum_log = atoi(argv[6]);
    const int fast_n = atoi(argv[7]);
    const int submitters = atoi(argv[8]);
    const int queue_cap = atoi(argv[9]);
    const std::string fault = argv[10];
    const int fault_at = atoi(argv[11]);
    const int n_lo = atoi(argv[12]), n_hi = atoi(argv[13]);
    const int timeout_ms = atoi(argv[14]);

    std::vector<std::vector<uint8_t>> mats((size_t)count);
    std::vector<int> ns((size_t)count);
    for (int k = 0; k < count; ++k) {
        const int n = k % 17 == 5 ? 0 : n_lo + (int)(splitmix(seed) % (uint64_t)(n_hi - n_lo + 1));
        ns[k] = n;
        mats[k].resize((size_t)n * n);
        for (auto &x : mats[k]) x = (uint8_t)(splitmix(seed) % 3);
    }

    SchedParams p;
    memset(&p.cfg, 0, sizeof p.cfg);
    p.cfg.max_slots = max_slots;
    p.cfg.queue_cap = queue_cap;
    p.cfg.work_budget = budget_log ? 1ull << budget_log : 0;
    p.cfg.quantum = 1ull << quantum_log;
    p.cfg.policy = policy;
    p.cfg.fast_max_n = fast_n;
    p.cfg.tick_timeout_ms = timeout_ms;
    p.fast_n = fast_n;
    p.max_tasks = sched_max_tasks(p.cfg);

    MockExecutor ex(max_slots);
    ex.budget = p.cfg.work_budget;
    if (fault == "launch") ex.fault = MockExecutor::LAUNCH;
    if (fault == "fast") ex.fault = MockExecutor::FAST;
    if (fault == "hang") ex.fault = MockExecutor::HANG;
    ex.fault_at = fault_at;

    int32_t fatal = PERM_OK;
    std::map<uint64_t, perm_done> got;
    perm_server_stats st{};
    {
        Scheduler sched(p, &ex);
        sched.start();
        std::atomic<bool> stop_poll{false};
        std::mutex got_mu;
        std::thread poller([&] {
            std::vector<perm_done> buf(256);
            while (!stop_poll.load()) {
                int32_t k = 0;
                sched.poll(buf.data(), (int32_t)buf.size(), &k, 2000);
                std::lock_guard<std::mutex> g(got_mu);
                for (int32_t i = 0; i < k; ++i) {
                    CHECK(got.count(buf[i].tag) == 0, "request %llu reported twice",
                          (unsigned long long)buf[i].tag);
                    got[buf[i].tag] = buf[i];
                }
            }
        });
        std::vector<std::thread> subs;
        for (int t = 0; t < submitters; ++t)
            subs.emplace_back([&, t] {
                for (int k = t; k < count; k += submitters) {
                    for (;;) {
                        const int32_t rc = sched.submit(mats[k].data(), ns[k], (uint64_t)k);
                        if (rc == PERM_OK) break;
                        if (rc == PERM_ESTATE) return;   // the server failed and stopped
                        CHECK(rc == PERM_EAGAIN, "submit returned %d", rc);
                        std::this_thread::sleep_for(std::chrono::microseconds(50));
                    }
                }
            });
        for (auto &th : subs) th.join();
        // wait until every accepted request has come back (each completes or, after a fault, fails)
        for (int spin = 0; spin < 600000; ++spin) {
            const perm_server_stats s = sched.stats();
            {
                std::lock_guard<std::mutex> g(got_mu);
                if (got.size() >= s.submitted) break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        fatal = sched.shutdown();
        stop_poll.store(true);
        poller.join();
        // anything published between the poller's last call and the shutdown
        std::vector<perm_done> buf(1024);
        int32_t k = 0;
        do {
            sched.poll(buf.data(), (int32_t)buf.size(), &k, 0);
            for (int32_t i = 0; i < k; ++i) got[buf[i].tag] = buf[i];
        } while (k > 0);
        st = sched.stats();
    }

    int ok_count = 0, failed = 0;
    for (auto &kv : got) {
        const perm_done &d = kv.second;
        const int k = (int)kv.first;
        CHECK(k >= 0 && k < count, "unknown tag %d", k);
        if (d.status == PERM_OK) {
            const int want = oracle_perm_mod3(mats[k].data(), ns[k], 1);
            CHECK(d.result == want, "request %d (n = %d): %d, oracle %d", k, ns[k], d.result, want);
            CHECK(d.n == ns[k], "request %d: n %d", k, d.n);
            CHECK(d.t_submit_ns <= d.t_admit_ns && d.t_admit_ns <= d.t_done_ns, "request %d: times out of order", k);
            ok_count++;
        } else {
            CHECK(d.status == PERM_EDEVICE, "request %d: status %d", k, d.status);
            failed++;
        }
    }
    if (fault == "none") {
        CHECK(fatal == PERM_OK, "shutdown returned %d", fatal);
        CHECK((int)got.size() == count, "%zu of %d requests came back", got.size(), count);
        CHECK(failed == 0, "%d requests failed", failed);
        CHECK((int)st.completed == count && (int)st.submitted == count, "stats: %llu submitted, %llu completed",
              (unsigned long long)st.submitted, (unsigned long long)st.completed);
    } else {
        CHECK(fatal == PERM_EDEVICE, "shutdown returned %d after a %s fault", fatal, fault.c_str());
        CHECK(failed > 0, "no request failed after a %s fault", fault.c_str());
        CHECK((int)got.size() == (int)st.submitted, "%zu of %llu accepted requests came back", got.size(),
              (unsigned long long)st.submitted);
    }
    CHECK(st.active_slots == 0 && st.queued == 0, "left: %d active, %d queued", st.active_slots, st.queued);
    printf("%s ok=%d failed=%d ticks=%llu launches=%d fast_calls=%d fatal=%d\n", g_errors ? "error" : "ok",
           ok_count, failed, (unsigned long long)st.ticks, ex.launches, ex.fast_calls, fatal);
    return g_errors ? 1 : 0;
}
