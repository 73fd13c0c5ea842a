// The serving scheduler under ThreadSanitizer, on the CPU fake executor.
//
// Four client threads submit requests of 1-700 rows for two forests while
// two threads poll their tickets and one reads statistics; every fourth
// launch fails and is retried; a small budget makes requests wait as heap
// copies.  Every result must equal the fake executor's row checksum (the
// scheduler moved the right rows in and the right votes out).  Exits 1 on a
// wrong result or status; ThreadSanitizer reports data races and exits 66.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "forest_file.h"
#include "forestpack.h"

static void fake_votes(const float* x, int F, int C, int32_t* out) {
    uint32_t h = 2166136261u;
    const uint8_t* b = reinterpret_cast<const uint8_t*>(x);
    for (int k = 0; k < F * 4; k++) h = (h ^ b[k]) * 16777619u;
    for (int c = 0; c < C; c++) out[c] = (int32_t)((h ^ ((uint32_t)c * 0x9E3779B9u)) & 0x7FFFFFFFu);
}

struct Req {
    int forest = 0;
    int64_t off = 0, rows = 0;
    std::vector<int32_t> out;
    uint64_t ticket = 0;
    std::atomic<int> posted{0};
};

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    ForestFile ff;
    if (!ff.read(argv[1])) return 2;
    const fp_forest_view v = ff.view();
    fp_packed* packs[2] = {nullptr, nullptr};
    fp_pack_opts po[2] = {{FP_LAYOUT_CLUSTERED, 4, 3, 0, FP_ORDER_DEFAULT}, {FP_LAYOUT_PACKED, 2, 2, 0, FP_ORDER_DEFAULT}};
    for (int i = 0; i < 2; i++)
        if (fp_pack_forest(&v, &po[i], &packs[i])) return 1;
    fp_server_opts o{};
    o.hbm_budget_bytes = 1 << 20;
    o.max_inflight = 3;
    o.max_rows_per_launch = 4096;
    o.max_retries = 4;
    o.executor = FP_EXECUTOR_CPU_FAKE;
    o.fake_delay_us = 30;
    o.fake_fail_every = 4;
    fp_server* s = nullptr;
    if (fp_server_create(&o, &s)) return 1;
    int32_t ids[2];
    for (int i = 0; i < 2; i++)
        if (fp_server_add_forest(s, packs[i], &ids[i])) return 1;
    const int F = ff.F, C = ff.C;
    const int64_t pool_rows = 30000;
    std::vector<float> pool((size_t)pool_rows * F);
    std::mt19937 rng(7);
    std::normal_distribution<float> nd;
    for (auto& x : pool) x = nd(rng);
    const int n_req = 1200, n_clients = 4;
    std::vector<Req> reqs(n_req);
    for (int i = 0; i < n_req; i++) {
        reqs[i].forest = (int)(rng() % 2);
        reqs[i].rows = 1 + (int64_t)(rng() % 700);
        reqs[i].off = (int64_t)(rng() % (uint32_t)(pool_rows - reqs[i].rows));
        reqs[i].out.assign((size_t)reqs[i].rows * C, -1);
    }
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int k = 0; k < n_clients; k++)
        th.emplace_back([&, k] {
            for (int i = k; i < n_req; i += n_clients) {
                Req& r = reqs[i];
                int rc;
                while ((rc = fp_serve_submit(s, ids[r.forest], pool.data() + r.off * F, r.rows, F, r.out.data(),
                                             &r.ticket)) == FP_EAGAIN)
                    std::this_thread::yield();
                if (rc) bad++;
                r.posted.store(1, std::memory_order_release);
            }
        });
    std::atomic<int> polled{0};
    for (int k = 0; k < 2; k++)
        th.emplace_back([&, k] {
            for (int i = k; i < n_req; i += 2) {
                Req& r = reqs[i];
                while (!r.posted.load(std::memory_order_acquire)) std::this_thread::yield();
                if (fp_serve_poll(s, r.ticket, -1) != FP_OK) bad++;
                polled++;
            }
        });
    std::atomic<bool> done{false};
    std::thread stats([&] {
        fp_serve_stats st;
        while (!done.load()) {
            if (fp_server_stats(s, &st)) bad++;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    for (auto& t : th) t.join();
    done = true;
    stats.join();
    fp_serve_stats st;
    fp_server_stats(s, &st);
    fp_server_destroy(s);
    std::vector<int32_t> want(C);
    for (const Req& r : reqs)
        for (int64_t i = 0; i < r.rows; i++) {
            fake_votes(pool.data() + (r.off + i) * F, F, C, want.data());
            if (memcmp(want.data(), r.out.data() + i * C, sizeof(int32_t) * C)) {
                bad++;
                break;
            }
        }
    for (auto* p : packs) fp_packed_free(p);
    printf("serve_tsan: %d requests, %d polled, %lld launches, %lld failed and retried, %d wrong\n", n_req,
           polled.load(), (long long)st.launches, (long long)st.failed_launches, bad.load());
    return bad.load() == 0 && st.failed_launches > 0 ? 0 : 1;
}
