// Concurrency stress of the continuous-batching server on its host-only
// timing backend (no device), for the thread and address/undefined sanitizer
// builds: several submitting threads, one thread that polls and releases,
// one that reads statistics, while the scheduler thread runs. Exit status 0
// when every request completes exactly once. Test infrastructure only.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "fe.h"

int main()
{
    fe_quad_rule r1{}, r6{};
    if (fe_quad_rule_builtin(FE_TET4, 1, &r1) || fe_quad_rule_builtin(FE_PRISM6, 6, &r6))
        return 90;
    fe_batch_kind kinds[2]{};
    kinds[0].problem.kind = FE_SCALAR_CDR;
    kinds[0].problem.precision = FE_FP64;
    kinds[0].problem.coef_mode = FE_COEF_PER_ELEMENT;
    kinds[0].problem.coef_mask = (1u << 20) - 1;
    kinds[0].problem.k_format = FE_K_FULL;
    kinds[0].elem_type = FE_TET4;
    kinds[0].n_q = r1.n_q;
    kinds[0].xi = r1.xi;
    kinds[0].w = r1.w;
    kinds[1].problem.kind = FE_ELASTICITY;
    kinds[1].problem.precision = FE_FP32_BULK;
    kinds[1].problem.coef_mode = FE_COEF_PER_ELEMENT;
    kinds[1].problem.coef_mask = 31;
    kinds[1].problem.k_format = FE_K_SYM_PACKED;
    kinds[1].elem_type = FE_PRISM6;
    kinds[1].n_q = r6.n_q;
    kinds[1].xi = r6.xi;
    kinds[1].w = r6.w;
    fe_server_config cfg{};
    cfg.kinds = kinds;
    cfg.n_kinds = 2;
    cfg.max_slots = 6;
    cfg.hbm_budget_bytes = 256ll << 20;
    cfg.max_chunks = 32;
    cfg.chunk_elems = 1024;
    cfg.backend = FE_SERVER_FAKE;
    cfg.fake_ns_per_elem = 0.5;
    cfg.fake_h2d_bytes_per_s = 200e9;
    cfg.fake_tick_overhead_s = 2e-6;
    fe_server *s = nullptr;
    if (fe_server_create(&cfg, &s) != FE_OK) {
        std::fprintf(stderr, "create: %s\n", fe_last_error());
        return 91;
    }
    static double dummy[64];  // the timing backend never reads inputs
    const int n_threads = 4, per_thread = 60;
    std::atomic<int> submitted{0}, too_big{0};
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t)
        th.emplace_back([&, t] {
            std::mt19937 g(1234 + t);
            for (int i = 0; i < per_thread; ++i) {
                fe_request rq{};
                rq.kind = (int)(g() % 2);
                rq.n_elem = 1 + (int64_t)(g() % 30000);
                if (i % 37 == 5)
                    rq.n_elem = 3000000;  // larger than the whole budget: fails alone
                rq.coords = dummy;
                rq.coeffs = dummy;
                rq.ld_in = rq.n_elem;
                rq.tag = (uint64_t)(t * per_thread + i);
                uint64_t id = 0;
                if (fe_server_submit(s, &rq, &id) == FE_OK) {
                    submitted.fetch_add(1);
                    if (rq.n_elem == 3000000)
                        too_big.fetch_add(1);
                }
            }
        });
    std::atomic<bool> done{false};
    std::set<uint64_t> seen;  // poller only
    std::atomic<int> ok{0}, failed{0}, dup{0};
    std::thread poller([&] {
        fe_completion c[16];
        while (!done.load() || ok + failed < submitted.load()) {
            const int n = fe_server_poll(s, c, 16, 0.01);
            for (int i = 0; i < n; ++i) {
                if (!seen.insert(c[i].id).second)
                    ++dup;
                if (c[i].status == FE_OK)
                    ok.fetch_add(1);
                else
                    failed.fetch_add(1);
                fe_server_release(s, c[i].id);
            }
            if (done.load() && ok + failed >= submitted.load())
                break;
        }
    });
    std::thread reader([&] {
        fe_server_stats st{};
        while (!done.load() || ok + failed < submitted.load()) {
            fe_server_stats_get(s, &st);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            if (done.load() && ok + failed >= submitted.load())
                break;
        }
    });
    for (auto &x : th)
        x.join();
    done.store(true);
    poller.join();
    reader.join();
    fe_server_stats st{};
    fe_server_stats_get(s, &st);
    fe_server_destroy(s);
    std::printf("server stress: submitted %d ok %d failed %d (expected %d) dup %d in use %lld\n",
                submitted.load(), ok.load(), failed.load(), too_big.load(), dup.load(),
                (long long)st.bytes_in_use);
    const bool good = ok + failed == submitted.load() && failed == too_big.load() && dup == 0 &&
                      st.bytes_in_use == 0 && submitted.load() == n_threads * per_thread;
    return good ? 0 : 1;
}
