// CPU emulation of the look-back protocol of the single-sweep radix passes
// (decoupled look-back over a chained scan): worker threads play the
// workgroups that are resident at one time, each tile publishes its count
// per digit (flag A), looks back over the tiles before it a few descriptors
// per load round, adding counts up to the first inclusive prefix (flag P),
// and publishes its own prefix.  Several passes share one descriptor array
// (flags 2p + 1 and 2p + 2, cleared once), as in one sort.
//
// Mode "ordered": tiles take their index from a counter in the order the
// workers start them (the kernel's scheme).  Every prefix must be exact and
// no wait may reach its bound, for fewer workers than tiles and random
// delays at every step.
//
// Mode "static": worker w takes tiles w, w + W, w + 2W, ... (a fixed
// assignment, as blockIdx would give with fewer resident workgroups than
// tiles, in an order the hardware does not promise).  A tile can then wait
// on a tile whose worker is itself waiting further up its own list; the
// bound is what ends such waits, and the run must still terminate.
//
// Usage: sort_lookback_emul ordered|static
// Prints one line "tiles_checked=N mismatches=M bound_hits=B"; exit 0.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr int kDigits = 8;

struct Run {
    int nb = 0, workers = 0, window = 2, passes = 8;
    uint32_t spin_bound = 1u << 22;
    bool ordered = true;
    std::vector<std::atomic<uint64_t>> desc;
    std::vector<uint32_t> cnt, got;
    std::atomic<int> ctr{0};
    std::atomic<long> bound_hits{0};
};

void delay(std::mt19937 &r) {
    if (r() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(r() % 100));
}

void tile_work(Run &R, int pass, int t, std::mt19937 &r) {
    const uint64_t fa = (uint64_t)(2 * pass + 1) << 32, fp = (uint64_t)(2 * pass + 2) << 32;
    delay(r);  // loading and ranking
    for (int d = 0; d < kDigits; ++d)
        R.desc[(size_t)t * kDigits + d].store((t == 0 ? fp : fa) | R.cnt[(size_t)t * kDigits + d],
                                             std::memory_order_relaxed);
    delay(r);  // staging in LDS
    for (int d = 0; d < kDigits; ++d) {
        uint32_t excl = 0;
        if (t > 0) {
            long k = t - 1;
            uint32_t spins = 0;
            for (;;) {
                std::vector<uint64_t> v(R.window);
                for (int u = 0; u < R.window; ++u)
                    v[u] = k - u >= 0 ? R.desc[(size_t)(k - u) * kDigits + d].load(
                                            std::memory_order_relaxed)
                                      : 0ull;
                int used = R.window;
                bool done = false;
                for (int u = 0; u < R.window; ++u) {
                    if (used != R.window || done) continue;
                    const uint32_t f = (uint32_t)(v[u] >> 32);
                    if (k - u < 0 || f < (uint32_t)(2 * pass + 1)) {
                        used = u;
                        continue;
                    }
                    excl += (uint32_t)v[u];
                    done = f == (uint32_t)(2 * pass + 2);
                }
                if (done) break;
                k -= used;
                if (used == 0) {
                    if (++spins >= R.spin_bound) {
                        R.bound_hits++;
                        break;
                    }
                    std::this_thread::yield();
                }
            }
            R.desc[(size_t)t * kDigits + d].store(fp | (uint64_t)(excl + R.cnt[(size_t)t * kDigits + d]),
                                                 std::memory_order_relaxed);
        }
        R.got[(size_t)t * kDigits + d] = excl;
    }
}

}  // namespace

int main(int argc, char **argv) {
    const bool ordered = argc < 2 || std::strcmp(argv[1], "static") != 0;
    long checked = 0, mismatches = 0, hits = 0;
    const int trials = ordered ? 24 : 4;
    for (int trial = 0; trial < trials; ++trial) {
        Run R;
        R.ordered = ordered;
        R.nb = ordered ? 1 + (trial * 53) % 400 : 64;
        R.workers = ordered ? 1 + trial % 9 : 4;
        R.window = 1 + trial % 4;
        R.passes = ordered ? 8 : 1;
        R.spin_bound = ordered ? (1u << 22) : 2000u;
        R.desc = std::vector<std::atomic<uint64_t>>((size_t)R.nb * kDigits);
        for (auto &x : R.desc) x.store(0);
        std::mt19937 g(trial);
        for (int pass = 0; pass < R.passes; ++pass) {
            R.cnt.assign((size_t)R.nb * kDigits, 0);
            for (auto &c : R.cnt) c = g() % 64;
            R.got.assign((size_t)R.nb * kDigits, 0xFFFFFFFFu);
            R.ctr.store(0);
            std::vector<std::thread> th;
            for (int w = 0; w < R.workers; ++w) {
                th.emplace_back([&R, pass, w, trial]() {
                    std::mt19937 r(trial * 1000 + pass * 31 + w);
                    if (R.ordered) {
                        for (;;) {
                            const int t = R.ctr.fetch_add(1);
                            if (t >= R.nb) return;
                            tile_work(R, pass, t, r);
                        }
                    } else {
                        // a worker takes its tiles from the top of its list,
                        // so lower tiles of other workers may not have started
                        for (int t = R.nb - R.workers + w; t >= 0; t -= R.workers)
                            tile_work(R, pass, t, r);
                    }
                });
            }
            for (auto &x : th) x.join();
            if (ordered) {
                for (int d = 0; d < kDigits; ++d) {
                    uint32_t run = 0;
                    for (int t = 0; t < R.nb; ++t) {
                        mismatches += R.got[(size_t)t * kDigits + d] != run;
                        ++checked;
                        run += R.cnt[(size_t)t * kDigits + d];
                    }
                }
            }
        }
        hits += R.bound_hits.load();
    }
    std::printf("tiles_checked=%ld mismatches=%ld bound_hits=%ld\n", checked, mismatches, hits);
    return 0;
}
