// Multi-threaded driver of the serving scheduler on the fake executor
// (fake_device.cpp): submitters, a poller that checks and releases results,
// a canceller, a statistics reader and fetches race with the scheduler
// thread; then a server is destroyed with requests still queued and running.
// Every result is checked exactly (the fake step adds 1 per step), the
// scheduler's admitted device memory is checked against its budget, and the
// process exits non-zero on any mismatch.  Built with -fsanitize=address,
// undefined or -fsanitize=thread by tests/test_serve_host.py.
//
//   serve_stress [requests] [seed]
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../include/pfmi.h"

extern "C" int64_t fake_model_bytes_peak(void);
extern "C" int64_t fake_model_bytes_live(void);
extern "C" void fake_device_idle(void);
extern "C" void fake_reset_peak(void);
extern "C" void fake_fail_creates(int every);

namespace {

std::atomic<int> g_fail{0};

void check(bool ok, const char *what, unsigned long long a = 0, unsigned long long b = 0)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (%llu, %llu)\n", what, a, b);
        g_fail++;
    }
}

struct Spec {
    pf_desc d;
    int64_t nsteps;
    uint64_t seed;
    int64_t sites;
};

Spec make_spec(std::mt19937_64 &rng, int i)
{
    Spec s{};
    pf_desc &d = s.d;
    std::memset(&d, 0, sizeof d);
    d.struct_size = sizeof(pf_desc);
    d.kind = 1 + (int)(rng() % 3);
    d.nfields = d.kind == PF_GS ? 2 : 1;
    d.ndim = 2 + (int)(rng() % 2);
    d.n[0] = 4 + (int64_t)(rng() % 29);
    d.n[1] = 4 + (int64_t)(rng() % 29);
    d.n[2] = d.ndim == 3 ? 2 + (int64_t)(rng() % 9) : 1;
    d.dx = 1.0;
    d.dt = 0.01;
    d.order = 2 + 2 * (int)(rng() % 2);
    d.precision = (int)(rng() % 2);
    d.nparams = d.kind == PF_GS ? 4 : 2;
    s.nsteps = (int64_t)(rng() % 7 == 0 ? 0 : rng() % 300);
    s.seed = 1000 * (uint64_t)i + rng() % 997;
    s.sites = d.n[0] * d.n[1] * d.n[2];
    return s;
}

// expected final state: field 0 = x0 + n, field 1 = x0 + 1 + n (fake step)
double expect_mass(const Spec &s, int f)
{
    const double x0 = (double)(s.seed % 1000) + f;
    return (double)s.sites * (x0 + (double)s.nsteps);
}

int run_mix(int nreq, uint64_t seed)
{
    // a budget of a few requests' footprints and few slots force queueing
    pf_server *srv = nullptr;
    const uint64_t budget = 300000;
    check(pf_server_create(0, budget, 6, 16, &srv) == PF_OK, "create");
    std::mutex mu;
    std::map<uint64_t, Spec> specs;
    std::set<uint64_t> cancelled;
    std::atomic<int> submitted{0}, done{0};
    std::atomic<bool> stop{false};
    const int nsub = 2;

    auto submitter = [&](int id) {
        std::mt19937_64 rng(seed * 31 + (uint64_t)id);
        for (int i = id; i < nreq; i += nsub) {
            Spec s = make_spec(rng, i);
            uint64_t t = 0;
            const pf_status st = pf_server_submit(srv, &s.d, PF_IC_UNIFORM, s.seed, nullptr, 0,
                                                  s.nsteps, &t);
            if (st == PF_ERR_NOMEM) {  // larger than the whole budget: refused up front
                check(pf_footprint_bytes(&s.d) > budget, "NOMEM for a request that fits");
                submitted++;
                done++;
                continue;
            }
            check(st == PF_OK, "submit", (unsigned long long)st);
            {
                std::lock_guard<std::mutex> lk(mu);
                specs[t] = s;
            }
            submitted++;
            if (rng() % 4 == 0) std::this_thread::yield();
        }
    };
    auto canceller = [&] {
        std::mt19937_64 rng(seed ^ 0xC0FFEE);
        while (!stop.load()) {
            uint64_t t = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!specs.empty() && rng() % 3 == 0) {
                    auto it = specs.begin();
                    std::advance(it, (long)(rng() % specs.size()));
                    t = it->first;
                    cancelled.insert(t);  // before the call: its result may come back at once
                }
            }
            if (t) {
                const pf_status st = pf_server_cancel(srv, t);
                // released tickets are unknown; the rest take the cancel
                check(st == PF_OK || st == PF_ERR_NOTFOUND, "cancel", (unsigned long long)st);
            }
            std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
    };
    auto stats_reader = [&] {
        int64_t last = 0;
        while (!stop.load()) {
            int64_t ticks = 0, l = 0, c = 0, r = 0;
            check(pf_server_stats(srv, &ticks, &l, &c, &r) == PF_OK, "stats");
            check(ticks >= last, "ticks went backwards");
            last = ticks;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    };

    std::vector<std::thread> th;
    for (int i = 0; i < nsub; ++i) th.emplace_back(submitter, i);
    th.emplace_back(canceller);
    th.emplace_back(stats_reader);

    // poller (this thread): check, sometimes fetch, release
    std::mt19937_64 rng(seed + 7);
    std::vector<pf_result> buf(64);
    while (done.load() < nreq) {
        int32_t n = 0;
        check(pf_server_poll(srv, buf.data(), (int32_t)buf.size(), &n) == PF_OK, "poll");
        for (int k = 0; k < n; ++k) {
            const pf_result &r = buf[k];
            Spec s;
            bool was_cancelled;
            for (;;) {  // the submitter records the spec just after submit returns
                std::lock_guard<std::mutex> lk(mu);
                if (specs.count(r.ticket)) {
                    s = specs[r.ticket];
                    was_cancelled = cancelled.count(r.ticket) != 0;
                    break;
                }
            }
            if (r.status == PF_OK) {
                check(r.steps_done == s.nsteps, "steps_done", (unsigned long long)r.steps_done,
                      (unsigned long long)s.nsteps);
                check(r.mass[0] == expect_mass(s, 0), "mass of field 0", r.ticket);
                if (s.d.nfields == 2) check(r.mass[1] == expect_mass(s, 1), "mass of field 1", r.ticket);
                check(r.t_submit <= r.t_admit && r.t_admit <= r.t_done, "timestamps", r.ticket);
                if (rng() % 5 == 0) {
                    std::vector<double> f((size_t)s.sites);
                    check(pf_server_fetch(srv, r.ticket, 0, f.data(), s.sites) == PF_OK, "fetch");
                    const double want = (double)(s.seed % 1000) + (double)s.nsteps;
                    for (double v : f) check(v == want, "fetched value", r.ticket);
                }
            } else {
                check(r.status == PF_ERR_STATE && was_cancelled, "failed without a cancel",
                      r.ticket, (unsigned long long)r.status);
                check(r.steps_done <= s.nsteps, "cancelled steps", r.ticket);
            }
            check(pf_server_release(srv, r.ticket) == PF_OK, "release", r.ticket);
            check(pf_server_release(srv, r.ticket) == PF_ERR_NOTFOUND, "second release", r.ticket);
            {
                std::lock_guard<std::mutex> lk(mu);
                specs.erase(r.ticket);
            }
            done++;
        }
        if (n == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    for (int i = 0; i < nsub; ++i) th[i].join();
    check(pf_server_drain(srv, 30.0) == PF_OK, "drain");
    stop = true;
    for (size_t i = nsub; i < th.size(); ++i) th[i].join();
    pf_server_destroy(srv);
    fake_device_idle();
    check(fake_model_bytes_peak() <= (int64_t)budget, "admitted memory above the budget",
          (unsigned long long)fake_model_bytes_peak(), budget);
    check(fake_model_bytes_live() == 0, "model memory leaked", (unsigned long long)fake_model_bytes_live());
    return 0;
}

// A queued request cancelled and released must not return budget it never
// took: the budget still bounds what is admitted afterwards.
int run_cancel_queued(uint64_t seed)
{
    pf_server *srv = nullptr;
    std::mt19937_64 rng(seed);
    pf_desc d{};
    d.struct_size = sizeof(pf_desc);
    d.kind = PF_AC;
    d.nfields = 1;
    d.ndim = 2;
    d.n[0] = 32;
    d.n[1] = 32;
    d.n[2] = 1;
    d.dx = 1.0;
    d.dt = 0.01;
    d.order = 2;
    d.nparams = 2;
    const uint64_t fp = pf_footprint_bytes(&d);
    const uint64_t budget = 2 * fp;  // two requests at a time
    fake_device_idle();
    const int64_t base = fake_model_bytes_live();
    fake_reset_peak();
    check(pf_server_create(0, budget, 16, 8, &srv) == PF_OK, "create");
    std::vector<uint64_t> t(8);
    for (int i = 0; i < 8; ++i)
        check(pf_server_submit(srv, &d, PF_IC_UNIFORM, 1 + i, nullptr, 0, 4000, &t[i]) == PF_OK, "submit");
    // the last ones are still queued behind the budget: cancel them, then
    // submit more behind them; finished requests hold their memory until
    // released, so release every result as it comes
    for (int i = 5; i < 8; ++i) check(pf_server_cancel(srv, t[i]) == PF_OK, "cancel");
    for (int i = 0; i < 4; ++i) {
        uint64_t x;
        check(pf_server_submit(srv, &d, PF_IC_UNIFORM, 50 + i, nullptr, 0, 100, &x) == PF_OK, "submit");
    }
    std::vector<pf_result> buf(16);
    int seen = 0, cancelled_seen = 0;
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::seconds(60);
    while (seen < 12 && std::chrono::steady_clock::now() < t_end) {
        int32_t n = 0;
        check(pf_server_poll(srv, buf.data(), 16, &n) == PF_OK, "poll");
        for (int k = 0; k < n; ++k) {
            cancelled_seen += buf[k].status == PF_ERR_STATE;
            check(pf_server_release(srv, buf[k].ticket) == PF_OK, "release");
            seen++;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    check(seen == 12 && cancelled_seen == 3, "results of the cancel test", (unsigned long long)seen,
          (unsigned long long)cancelled_seen);
    check(pf_server_drain(srv, 10.0) == PF_OK, "drain");
    fake_device_idle();
    check(fake_model_bytes_peak() - base <= (int64_t)budget, "cancelled queued request freed budget",
          (unsigned long long)(fake_model_bytes_peak() - base), budget);
    pf_server_destroy(srv);
    (void)rng;
    return 0;
}

// Allocation failures at admission: every third model creation fails.  Those
// requests come back with PF_ERR_NOMEM and no steps, every other one is
// exact, and no memory or budget leaks.
int run_alloc_failures(uint64_t seed)
{
    std::mt19937_64 rng(seed + 11);
    pf_server *srv = nullptr;
    const uint64_t budget = 400000;
    fake_device_idle();
    fake_reset_peak();
    check(pf_server_create(0, budget, 8, 16, &srv) == PF_OK, "create");
    fake_fail_creates(3);
    const int nreq = 90;
    std::map<uint64_t, Spec> specs;
    for (int i = 0; i < nreq; ++i) {
        Spec s = make_spec(rng, i);
        uint64_t t = 0;
        check(pf_server_submit(srv, &s.d, PF_IC_UNIFORM, s.seed, nullptr, 0, s.nsteps, &t) == PF_OK, "submit");
        specs[t] = s;
    }
    std::vector<pf_result> buf(32);
    int seen = 0, nomem = 0;
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::seconds(60);
    while (seen < nreq && std::chrono::steady_clock::now() < t_end) {
        int32_t n = 0;
        check(pf_server_poll(srv, buf.data(), (int32_t)buf.size(), &n) == PF_OK, "poll");
        for (int k = 0; k < n; ++k) {
            const pf_result &r = buf[k];
            const Spec &s = specs[r.ticket];
            if (r.status == PF_ERR_NOMEM) {
                nomem++;
                check(r.steps_done == 0, "failed request advanced", r.ticket);
            } else {
                check(r.status == PF_OK, "status", r.ticket, (unsigned long long)r.status);
                check(r.steps_done == s.nsteps && r.mass[0] == expect_mass(s, 0), "result of a healthy request",
                      r.ticket);
            }
            check(pf_server_release(srv, r.ticket) == PF_OK, "release", r.ticket);
            seen++;
        }
        if (n == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    check(seen == nreq && nomem == nreq / 3, "injected failures", (unsigned long long)seen,
          (unsigned long long)nomem);
    check(pf_server_drain(srv, 10.0) == PF_OK, "drain");
    pf_server_destroy(srv);
    fake_fail_creates(0);
    fake_device_idle();
    check(fake_model_bytes_peak() <= (int64_t)budget, "admitted memory above the budget",
          (unsigned long long)fake_model_bytes_peak(), budget);
    check(fake_model_bytes_live() == 0, "model memory leaked after failures",
          (unsigned long long)fake_model_bytes_live());
    return 0;
}

// Destroy with a backlog: requests queued, running and finished-unreleased.
int run_destroy_backlog(uint64_t seed)
{
    std::mt19937_64 rng(seed);
    for (int round = 0; round < 5; ++round) {
        pf_server *srv = nullptr;
        check(pf_server_create(0, 200000, 4, 8, &srv) == PF_OK, "create");
        for (int i = 0; i < 40; ++i) {
            Spec s = make_spec(rng, i);
            uint64_t t;
            const pf_status st = pf_server_submit(srv, &s.d, PF_IC_UNIFORM, s.seed, nullptr, 0,
                                                  s.nsteps, &t);
            check(st == PF_OK || st == PF_ERR_NOMEM, "submit");
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(round));
        pf_server_destroy(srv);
    }
    fake_device_idle();
    check(fake_model_bytes_live() == 0, "model memory leaked after destroy",
          (unsigned long long)fake_model_bytes_live());
    return 0;
}

}  // namespace

int main(int argc, char **argv)
{
    const int nreq = argc > 1 ? std::atoi(argv[1]) : 400;
    const uint64_t seed = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1;
    run_mix(nreq, seed);
    run_cancel_queued(seed);
    run_alloc_failures(seed);
    run_destroy_backlog(seed);
    if (g_fail.load()) {
        std::fprintf(stderr, "serve_stress: %d failures\n", g_fail.load());
        return 1;
    }
    std::printf("serve_stress: ok (%d requests)\n", nreq);
    return 0;
}
