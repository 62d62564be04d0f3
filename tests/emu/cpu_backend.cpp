// Test-only CPU backend: runs the planner's grouped jobs with plain loops so
// the Chief's bookkeeping (Step 1 / 2 / 3, the append orders, the
// UpdateRowTrafo case table) can be checked against the oracle without a GPU.
// It is linked only into tests/emu/_build/libgfech_emu.so, which nothing but
// the CPU tests loads; the product library links the HIP backend instead.
//
// The ECH here follows the same column-by-column elimination the GPU kernel
// uses (first not-yet-selected non-zero row of each column becomes its pivot,
// rows kept reduced in the negative form, transformation columns kept only
// for selected rows), so it checks that algorithm as well.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../paper_1806_04211_amd/csrc/backend.h"

namespace gfech {
namespace {

class CpuBackend final : public Backend {
public:
    const char* name() const override { return "cpu-emulator"; }
    // fresh memory holds garbage, as device memory does: the planner must zero what it relies on
    void* alloc(size_t bytes) override {
        void* p = malloc(bytes ? bytes : 1);
        if (p) {
            memset(p, 0xA5, bytes ? bytes : 1);
            std::lock_guard<std::mutex> lk(allocs_mu());
            allocs()[(uintptr_t)p] = bytes;
        }
        return p;
    }
    void release(void* p) override {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(allocs_mu());
            allocs().erase((uintptr_t)p);
        }
        std::lock_guard<std::mutex> lk(quarantine_mu_);
        if (fuzz_) quarantine_.push_back(p);
        else free(p);
    }
    void zero(void* p, size_t bytes) override {
        if (fuzz_) { on_lane0([this, p, bytes] { if (bytes && chk(p, bytes, "zero")) memset(p, 0, bytes); }); return; }
        if (bytes && chk(p, bytes, "zero")) memset(p, 0, bytes);
    }
    void upload(void* dst, const void* src, size_t bytes) override {
        if (fuzz_) {
            std::vector<uint8_t> data((const uint8_t*)src, (const uint8_t*)src + bytes);
            on_lane0([this, dst, bytes, data] { if (bytes && chk(dst, bytes, "upload")) memcpy(dst, data.data(), bytes); });
            return;
        }
        if (bytes && chk(dst, bytes, "upload")) memcpy(dst, src, bytes);
    }
    void download(void* dst, const void* src, size_t bytes) override {
        if (fuzz_) drain(0, q_[0].size());
        if (bytes && chk(src, bytes, "download")) memcpy(dst, src, bytes);
    }
    void copy(void* dst, const void* src, size_t bytes) override {
        if (fuzz_) {
            on_lane0([this, dst, src, bytes] {
                if (bytes && chk(dst, bytes, "copy") && chk(src, bytes, "copy")) memmove(dst, src, bytes);
            });
            return;
        }
        if (bytes && chk(dst, bytes, "copy") && chk(src, bytes, "copy")) memmove(dst, src, bytes);
    }
    // Lanes: the jobs of lanes 1, 2 and 3 are queued and run as late as the
    // planner's marks allow (when lane 0 waits for them, when a queued wait of
    // another lane needs them, or at sync).  Any job the planner ordered
    // wrongly across the lanes then reads or overwrites data out of turn, and
    // the results stop matching the oracle.  GFECH_EMU_EAGER=1 runs
    // everything at once instead.  A mark is (queue length << 2) | lane; lane
    // 0's work is always complete, so its marks are 0.
    //
    // Fuzz mode (gfech_emu_set_fuzz(seed), seed != 0): lane 0 is queued as
    // well, and the queued jobs of all four lanes run in a seeded random
    // interleaving that respects only the order within a lane and the
    // recorded waits.  Memory transfers are lane-0 jobs; a download (and so
    // the read of the pivot counts) waits for lane 0 alone, as on the device.
    // A wait missing in either direction (a lane-0 job that needs earlier
    // work of lanes 1-3, or a job of lanes 1-3 that needs earlier lane-0
    // work) then lets a job run out of turn for some seeds.  Released memory
    // is quarantined until every queue is empty, so a queued job that touches
    // a buffer after its release fails the bounds check instead of landing in
    // a new allocation.
    // the fixed workspace: one allocation made once and never released
    uint8_t* fixed_scratch() override {
        if (!fixed_) fixed_ = (uint8_t*)alloc(kFixedScratchBytes);
        return fixed_;
    }
    void sync_lane0() override {
        if (fuzz_) drain(0, q_[0].size());
    }
    void set_lane(int lane) override { lane_ = lane; }
    int mark(int lane) override {
        if (lane == 0 && !fuzz_) return 0;
        return (int)((q_[lane].size() << 2) | (size_t)lane);
    }
    void wait_mark(int lane, int m) override {
        const int src = m & 3;
        const size_t upto = (size_t)(m >> 2);
        if (lane == drop_lane_ && src == drop_src_) return;   // a planted ordering mistake (tests only)
        if (fuzz_) {
            if (src == lane || upto == 0) return;
            Job j;
            j.wait_lane = src;
            j.wait_upto = upto;
            q_[lane].push_back(std::move(j));
            churn();
            return;
        }
        if (src == 0 || src == lane) return;
        if (lane == 0 || !defer_) drain(src, upto);
        else {
            Job j;
            j.f = [this, src, upto] { drain(src, upto); };
            q_[lane].push_back(std::move(j));
        }
    }
    void drain(int lane, size_t upto) {
        if (fuzz_) {
            while (done_[lane] < upto && done_[lane] < q_[lane].size()) {
                if (!step_random()) {
                    if (!err_) fprintf(stderr, "emulator: lanes wait for each other\n");
                    err_ = 6;
                    return;
                }
            }
            return;
        }
        while (done_[lane] < upto && done_[lane] < q_[lane].size()) {
            auto f = std::move(q_[lane][done_[lane]].f);
            ++done_[lane];
            f();
        }
    }
    void sync() override {
        while (done_[0] < q_[0].size() || done_[1] < q_[1].size() || done_[2] < q_[2].size() ||
               done_[3] < q_[3].size()) {
            if (fuzz_) {
                if (!step_random()) {
                    if (!err_) fprintf(stderr, "emulator: lanes wait for each other\n");
                    err_ = 6;
                    break;
                }
                continue;
            }
            drain(1, q_[1].size());
            drain(2, q_[2].size());
            drain(3, q_[3].size());
        }
        std::lock_guard<std::mutex> lk(quarantine_mu_);
        for (void* p : quarantine_) free(p);
        quarantine_.clear();
    }
    void drop_waits(int lane, int src) {
        drop_lane_ = lane;
        drop_src_ = src;
    }
    void set_fuzz(uint64_t seed) {
        sync();
        fuzz_ = seed != 0;
        rng_ = seed * 0x9E3779B97F4A7C15ull + 1;
    }
    int error() const override { return err_; }

    // every byte a job touches must lie inside one live allocation
    bool chk(const void* p, size_t bytes, const char* what) {
        if (bytes == 0) return true;
        uintptr_t a = (uintptr_t)p;
        {
            std::lock_guard<std::mutex> lk(allocs_mu());
            auto it = allocs().upper_bound(a);
            if (it != allocs().begin()) {
                --it;
                if (a >= it->first && a + bytes <= it->first + it->second) return true;
            }
        }
        if (!err_) fprintf(stderr, "emulator: out-of-bounds access in %s (%zu bytes at %p)\n", what, bytes, p);
        err_ = 6;
        return false;
    }
    bool gemm_ok(const GemmDesc& g) {
        bool ok = chk(g.D, 1, "gemm D");
        if (g.brow) ok &= chk(g.brow, sizeof(int32_t) * g.K, "gemm brow");
        if (g.crow) ok &= chk(g.crow, sizeof(int32_t) * g.M, "gemm crow");
        if (!ok) return false;
        for (int x = 0; x < g.M; ++x) {
            ok &= chk(g.D + (int64_t)x * g.ldd, g.N, "gemm D row");
            if (g.K) ok &= chk(g.A + (int64_t)x * g.lda, g.K, "gemm A row");
            if (g.C) ok &= chk(g.C + (int64_t)(g.crow ? g.crow[x] : x) * g.ldc, g.N, "gemm C row");
        }
        for (int k = 0; k < g.K; ++k) ok &= chk(g.B + (int64_t)(g.brow ? g.brow[k] : k) * g.ldb, g.N, "gemm B row");
        return ok;
    }

    void gemm(const std::vector<GemmDesc>& ds) override {
        enqueue([this, ds] { gemm_now(ds); });
    }
    void gemm_now(const std::vector<GemmDesc>& ds) {
        for (const GemmDesc& g : ds) {
            if (g.M <= 0 || g.N <= 0 || !gemm_ok(g)) continue;
            std::vector<uint8_t> out((size_t)g.M * g.N);
            for (int x = 0; x < g.M; ++x)
                for (int y = 0; y < g.N; ++y) {
                    uint64_t acc = 0;
                    if (g.C) {
                        int64_t cr = g.crow ? g.crow[x] : x;
                        acc = g.C[cr * g.ldc + y];
                    }
                    for (int k = 0; k < g.K; ++k) {
                        int64_t br = g.brow ? g.brow[k] : k;
                        acc += (uint64_t)g.A[(int64_t)x * g.lda + k] * g.B[br * g.ldb + y];
                    }
                    out[(size_t)x * g.N + y] = (uint8_t)(acc % (uint64_t)g.p);
                }
            for (int x = 0; x < g.M; ++x) memcpy(g.D + (int64_t)x * g.ldd, &out[(size_t)x * g.N], g.N);
        }
    }

    void gather(const std::vector<GatherDesc>& ds) override {
        enqueue([this, ds] { gather_now(ds); });
    }
    void gather_now(const std::vector<GatherDesc>& ds) {
        for (const GatherDesc& g : ds) {
            bool ok = true;
            if (g.srow) ok &= chk(g.srow, sizeof(int32_t) * g.rows, "gather srow");
            if (g.scol) ok &= chk(g.scol, sizeof(int32_t) * g.cols, "gather scol");
            if (g.drow) ok &= chk(g.drow, sizeof(int32_t) * g.rows, "gather drow");
            if (g.dcol) ok &= chk(g.dcol, sizeof(int32_t) * g.cols, "gather dcol");
            for (int x = 0; ok && x < g.rows; ++x)
                for (int y = 0; ok && y < g.cols; ++y) {
                    int64_t sr = g.srow ? g.srow[x] : x, sc = g.scol ? g.scol[y] : y;
                    int64_t dr = g.drow ? g.drow[x] : x, dc = g.dcol ? g.dcol[y] : y;
                    ok &= chk(g.src + sr * g.lds + sc, 1, "gather src") && chk(g.dst + dr * g.ldd + dc, 1, "gather dst");
                }
            if (!ok) continue;
            std::vector<uint8_t> tmp((size_t)g.rows * g.cols);
            for (int x = 0; x < g.rows; ++x)
                for (int y = 0; y < g.cols; ++y) {
                    int64_t sr = g.srow ? g.srow[x] : x, sc = g.scol ? g.scol[y] : y;
                    uint32_t v = g.src[sr * g.lds + sc];
                    if (g.neg_p) v = (g.neg_p - v) % g.neg_p;
                    tmp[(size_t)x * g.cols + y] = (uint8_t)v;
                }
            for (int x = 0; x < g.rows; ++x)
                for (int y = 0; y < g.cols; ++y) {
                    int64_t dr = g.drow ? g.drow[x] : x, dc = g.dcol ? g.dcol[y] : y;
                    g.dst[dr * g.ldd + dc] = tmp[(size_t)x * g.cols + y];
                }
        }
    }

    void fill(const std::vector<FillDesc>& ds) override {
        enqueue([this, ds] { fill_now(ds); });
    }
    void fill_now(const std::vector<FillDesc>& ds) {
        for (const FillDesc& f : ds) {
            bool ok = true;
            if (f.dcol) {
                ok &= chk(f.dcol, sizeof(int32_t) * f.rows, "fill dcol");
                for (int t = 0; ok && t < f.rows; ++t) ok &= chk(f.dst + (int64_t)t * f.ldd + f.dcol[t], 1, "fill");
            } else {
                for (int x = 0; ok && x < f.rows; ++x) ok &= chk(f.dst + (int64_t)x * f.ldd, f.cols, "fill row");
            }
            if (!ok) continue;
            if (f.dcol) {
                for (int t = 0; t < f.rows; ++t) f.dst[(int64_t)t * f.ldd + f.dcol[t]] = (uint8_t)f.diag_value;
                continue;
            }
            for (int x = 0; x < f.rows; ++x)
                for (int y = 0; y < f.cols; ++y)
                    f.dst[(int64_t)x * f.ldd + y] = (uint8_t)((x == y && f.diag_value >= 0) ? f.diag_value : f.value);
        }
    }

    void lists(const std::vector<ListDesc>& ds) override {
        enqueue([this, ds] { lists_now(ds); });
    }
    void lists_now(const std::vector<ListDesc>& ds) {
        for (const ListDesc& l : ds) {
            bool ok = true;
            if (l.npick) {
                ok &= chk(l.append, sizeof(int32_t) * l.npick, "list append");
                if (l.pick) ok &= chk(l.pick, sizeof(int32_t) * l.npick, "list pick");
                if (l.map)
                    for (int t = 0; ok && t < l.npick; ++t) ok &= chk(l.map + (l.pick ? l.pick[t] : t), 4, "list map");
            }
            if (l.nkeep) {
                ok &= chk(l.keep_out, sizeof(int32_t) * l.nkeep, "list keep_out");
                if (l.keep) ok &= chk(l.keep, sizeof(int32_t) * l.nkeep, "list keep");
                if (l.map)
                    for (int t = 0; ok && t < l.nkeep; ++t) ok &= chk(l.map + (l.keep ? l.keep[t] : t), 4, "list map");
            }
            if (!ok) continue;
            for (int t = 0; t < l.npick; ++t) {
                const int u = l.pick ? l.pick[t] : t;
                l.append[t] = l.add + (l.map ? l.map[u] : u);
            }
            for (int s = 0; s < l.nkeep; ++s) {
                const int u = l.keep ? l.keep[s] : s;
                l.keep_out[s] = l.map ? l.map[u] : u;
            }
        }
    }

    void sort(const std::vector<SortDesc>& ds) override {
        enqueue([this, ds] { sort_now(ds); });
    }
    void sort_now(const std::vector<SortDesc>& ds) {
        for (const SortDesc& s : ds) {
            if (!chk(s.vals, sizeof(int32_t) * s.n, "sort vals") || !chk(s.out, sizeof(int32_t) * s.n, "sort out"))
                continue;
            for (int t = 0; t < s.n; ++t) {
                int rank = 0;
                for (int u = 0; u < s.n; ++u) rank += s.vals[u] < s.vals[t];
                s.out[rank] = s.add + (s.mode ? t : s.vals[t]);
            }
        }
    }

    void mad_gf2(const Gf2MadDesc& d) override {
        enqueue([this, d] {
            const int64_t wn = (d.N + 63) / 64;
            for (int64_t i = 0; i < d.M; ++i) {
                if (!chk(d.D + i * d.ldd, 8 * (size_t)wn, "gf2 mad D") ||
                    !chk(d.A + i * d.lda, 8 * (size_t)((d.K + 63) / 64), "gf2 mad A") ||
                    (d.C && !chk(d.C + i * d.ldc, 8 * (size_t)wn, "gf2 mad C")))
                    return;
                std::vector<uint64_t> o(wn, 0);
                if (d.C) for (int64_t w = 0; w < wn; ++w) o[w] = d.C[i * d.ldc + w];
                for (int64_t k = 0; k < d.K; ++k)
                    if ((d.A[i * d.lda + k / 64] >> (k % 64)) & 1u) {
                        if (!chk(d.B + k * d.ldb, 8 * (size_t)wn, "gf2 mad B")) return;
                        for (int64_t w = 0; w < wn; ++w) o[w] ^= d.B[k * d.ldb + w];
                    }
                for (int64_t w = 0; w < wn; ++w) d.D[i * d.ldd + w] = o[w];
            }
        });
    }
    // a lane-0 job, like the memory transfers
    void unpack_gf2(const uint64_t* src, int64_t m, int64_t n, int64_t ldw, uint8_t* dst, int64_t ldd) override {
        auto run = [this, src, m, n, ldw, dst, ldd] {
            for (int64_t x = 0; x < m; ++x) {
                if (!chk(src + x * ldw, 8 * (size_t)((n + 63) / 64), "unpack src") ||
                    !chk(dst + x * ldd, (size_t)n, "unpack dst"))
                    return;
                for (int64_t y = 0; y < n; ++y) dst[x * ldd + y] = (uint8_t)((src[x * ldw + y / 64] >> (y % 64)) & 1u);
            }
        };
        if (fuzz_) on_lane0(run);
        else run();
    }
    int64_t count_gf2_pad(const uint64_t* src, int64_t m, int64_t n, int64_t ldw) override {
        if (fuzz_) drain(0, q_[0].size());
        int64_t bad = 0;
        if (n % 64 == 0) return 0;
        for (int64_t x = 0; x < m; ++x)
            for (int64_t y = n; y < (n + 63) / 64 * 64; ++y) bad += (src[x * ldw + y / 64] >> (y % 64)) & 1u;
        return bad;
    }
    int64_t count_out_of_range(const uint8_t* A, int64_t m, int64_t n, int64_t lda, int32_t p) override {
        if (fuzz_) drain(0, q_[0].size());
        int64_t bad = 0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) bad += A[i * lda + j] >= p;
        return bad;
    }

    void ech(const std::vector<EchDesc>& ds) override {
        enqueue([this, ds] { ech_now(ds); });
    }
    void ech_now(const std::vector<EchDesc>& ds) {
        for (const EchDesc& e : ds) {
            const int maxr = e.rows < e.cols ? e.rows : e.cols;
            bool ok = chk(e.rcount, 4, "ech rcount") && chk(e.prow, 4 * maxr, "ech prow") &&
                      chk(e.pcol, 4 * maxr, "ech pcol") && chk(e.qrow, 4 * e.rows, "ech qrow") &&
                      chk(e.qcol, 4 * e.cols, "ech qcol");
            for (int x = 0; ok && x < e.rows; ++x)
                ok &= chk(e.H + (int64_t)x * e.ldh, e.cols, "ech H") &&
                      chk(e.work + (int64_t)x * e.ldw, e.cols + maxr, "ech work");
            // outputs sized for the largest possible rank (what the kernel may write)
            for (int t = 0; ok && t < maxr; ++t) ok &= chk(e.Mo + (int64_t)t * e.ldm, maxr, "ech M");
            if (ok) {
                ech_one(e);
                int r = *e.rcount;
                for (int t = 0; ok && t < r; ++t) ok &= chk(e.Ro + (int64_t)t * e.ldr, e.cols - r, "ech R");
                for (int t = 0; ok && t < e.rows - r; ++t) ok &= chk(e.Ko + (int64_t)t * e.ldk, r, "ech K");
            }
        }
    }

private:
    // a queued job: work to run, or a wait for lane wait_lane to have run
    // wait_upto of its jobs (fuzz mode)
    struct Job {
        std::function<void()> f;
        int wait_lane = -1;
        size_t wait_upto = 0;
    };
    // live allocations of every instance (device memory is one address space:
    // a server's instances use each other's buffers)
    static std::map<uintptr_t, size_t>& allocs() {
        static std::map<uintptr_t, size_t> m;
        return m;
    }
    static std::mutex& allocs_mu() {
        static std::mutex mu;
        return mu;
    }
    uint8_t* fixed_ = nullptr;
    int err_ = 0;
    int lane_ = 0;
    bool defer_ = !(getenv("GFECH_EMU_EAGER") && getenv("GFECH_EMU_EAGER")[0] == '1');
    bool fuzz_ = false;
    int drop_lane_ = -1, drop_src_ = -1;
    uint64_t rng_ = 1;
    std::vector<Job> q_[4];
    size_t done_[4] = {0, 0, 0, 0};
    std::vector<void*> quarantine_;
    std::mutex quarantine_mu_;      // release() may run on another thread (a result freed there)
    uint64_t steps_ = 0;
    uint32_t weight_[4] = {1, 1, 1, 1};

    uint64_t next_rand() {   // xorshift64*
        rng_ ^= rng_ >> 12;
        rng_ ^= rng_ << 25;
        rng_ ^= rng_ >> 27;
        return rng_ * 0x2545F4914F6CDD1Dull;
    }
    void enqueue(std::function<void()> f) {
        if (fuzz_ || (lane_ != 0 && defer_)) {
            Job j;
            j.f = std::move(f);
            q_[lane_].push_back(std::move(j));
            if (fuzz_) churn();
            return;
        }
        f();
    }
    void on_lane0(std::function<void()> f) {
        Job j;
        j.f = std::move(f);
        q_[0].push_back(std::move(j));
        churn();
    }
    bool runnable(int lane) const {
        if (done_[lane] >= q_[lane].size()) return false;
        const Job& j = q_[lane][done_[lane]];
        return j.wait_lane < 0 || done_[j.wait_lane] >= j.wait_upto;
    }
    // run the head of a random lane that can proceed; false if none can.
    // Lanes are picked with weights (1, 8 or 64, re-drawn every 64 steps), so
    // that a lane may lag the others by several layers for a while.
    bool step_random() {
        if (steps_++ % 64 == 0)
            for (int l = 0; l < 4; ++l) weight_[l] = 1u << (3 * (next_rand() % 3));
        int cand[4], nc = 0;
        uint64_t total = 0;
        for (int l = 0; l < 4; ++l)
            if (runnable(l)) { cand[nc++] = l; total += weight_[l]; }
        if (!nc) return false;
        uint64_t x = next_rand() % total;
        int l = cand[0];
        for (int c = 0; c < nc; ++c) {
            if (x < weight_[cand[c]]) { l = cand[c]; break; }
            x -= weight_[cand[c]];
        }
        Job j = std::move(q_[l][done_[l]]);
        ++done_[l];
        if (j.f) j.f();
        return true;
    }
    // after every enqueue in fuzz mode: usually nothing (jobs stay queued
    // until a download or a sync forces them, so that many jobs of several
    // lanes are runnable together), sometimes a few random steps
    void churn() {
        if (next_rand() % 8 != 0) return;
        const int k = 1 + (int)(next_rand() % 3);
        for (int t = 0; t < k; ++t) if (!step_random()) break;
    }

    static uint32_t inv(uint32_t a, uint32_t p) {   // a^(p-2)
        uint32_t r = 1, b = a % p, x = p - 2;
        while (x) { if (x & 1) r = r * b % p; b = b * b % p; x >>= 1; }
        return r;
    }

    // work = [W | T] with W (rows x cols) the eliminated copy of H and T the
    // transformation columns of the selected rows (pivot order)
    void ech_one(const EchDesc& e) {
        const int rows = e.rows, cols = e.cols;
        const uint32_t p = (uint32_t)e.p;
        const int maxr = rows < cols ? rows : cols;
        for (int x = 0; x < rows; ++x) {
            memcpy(e.work + (int64_t)x * e.ldw, e.H + (int64_t)x * e.ldh, cols);
            memset(e.work + (int64_t)x * e.ldw + cols, 0, maxr);
        }
        auto W = [&](int x, int y) -> uint8_t& { return e.work[(int64_t)x * e.ldw + y]; };
        std::vector<char> selected(rows, 0);
        std::vector<int> prow, pcol;
        int r = 0;
        for (int c = 0; c < cols && r < maxr; ++c) {
            int piv = -1;
            for (int x = 0; x < rows; ++x)
                if (!selected[x] && W(x, c)) { piv = x; break; }
            if (piv < 0) continue;
            // scale the pivot row so the pivot becomes -1; its own transformation column is r
            uint32_t s = (p - inv(W(piv, c), p)) % p;
            W(piv, cols + r) = 1;
            for (int y = c; y < cols; ++y) W(piv, y) = (uint8_t)(W(piv, y) * s % p);
            for (int t = 0; t <= r; ++t) W(piv, cols + t) = (uint8_t)(W(piv, cols + t) * s % p);
            // clear column c in every other row: row += f * pivot row (pivot is -1)
            for (int x = 0; x < rows; ++x) {
                if (x == piv) continue;
                uint32_t f = W(x, c);
                if (!f) continue;
                for (int y = c; y < cols; ++y) W(x, y) = (uint8_t)((W(x, y) + f * W(piv, y)) % p);
                for (int t = 0; t <= r; ++t) W(x, cols + t) = (uint8_t)((W(x, cols + t) + f * W(piv, cols + t)) % p);
            }
            selected[piv] = 1;
            prow.push_back(piv);
            pcol.push_back(c);
            ++r;
        }
        *e.rcount = r;
        std::vector<char> pc(cols, 0);
        for (int t = 0; t < r; ++t) { e.prow[t] = prow[t]; e.pcol[t] = pcol[t]; pc[pcol[t]] = 1; }
        int q = 0;
        for (int x = 0; x < rows; ++x) if (!selected[x]) e.qrow[q++] = x;
        q = 0;
        for (int y = 0; y < cols; ++y) if (!pc[y]) e.qcol[q++] = y;
        for (int y = 0; y < e.qtail; ++y) e.qcol[q + y] = cols + y;
        // outputs
        for (int t = 0; t < r; ++t) {
            for (int u = 0; u < r; ++u) e.Mo[(int64_t)t * e.ldm + u] = W(prow[t], cols + u);
            int k = 0;
            for (int y = 0; y < cols; ++y) if (!pc[y]) e.Ro[(int64_t)t * e.ldr + k++] = W(prow[t], y);
        }
        q = 0;
        for (int x = 0; x < rows; ++x) {
            if (selected[x]) continue;
            for (int u = 0; u < r; ++u) e.Ko[(int64_t)q * e.ldk + u] = W(x, cols + u);
            ++q;
        }
    }
};

CpuBackend& instance() {
    static CpuBackend be;
    return be;
}

// the extra instances (server size classes), pooled and never destroyed;
// the test hooks below apply to every instance
std::mutex g_pool_mu;
std::vector<CpuBackend*> g_all, g_pool;
uint64_t g_fuzz_seed = 0;
int g_drop_lane = -1, g_drop_src = -1;

}  // namespace

Backend* backend_instance(std::string* err) {
    (void)err;
    return &instance();
}

Backend* backend_acquire(std::string* err) {
    (void)err;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool.empty()) {
        CpuBackend* b = g_pool.back();
        g_pool.pop_back();
        return b;
    }
    CpuBackend* b = new CpuBackend();
    // each instance draws its own interleaving from the seed
    b->set_fuzz(g_fuzz_seed ? g_fuzz_seed + 7919 * (g_all.size() + 1) : 0);
    b->drop_waits(g_drop_lane, g_drop_src);
    g_all.push_back(b);
    return b;
}

void backend_release(Backend* be) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(static_cast<CpuBackend*>(be));
}

}  // namespace gfech

// Test hook of the emulator build only: seed != 0 switches the randomized
// interleaving of all four lanes on (0 switches it off), for every instance.
extern "C" void gfech_emu_set_fuzz(uint64_t seed) {
    std::lock_guard<std::mutex> lk(gfech::g_pool_mu);
    gfech::g_fuzz_seed = seed;
    gfech::instance().set_fuzz(seed);
    for (size_t i = 0; i < gfech::g_all.size(); ++i)
        gfech::g_all[i]->set_fuzz(seed ? seed + 7919 * (i + 1) : 0);
}
// Test hook: ignore every wait of `lane` for work of lane `src` (-1: none), a
// planted ordering mistake that the randomized interleaving must expose.
extern "C" void gfech_emu_drop_waits(int lane, int src) {
    std::lock_guard<std::mutex> lk(gfech::g_pool_mu);
    gfech::g_drop_lane = lane;
    gfech::g_drop_src = src;
    gfech::instance().drop_waits(lane, src);
    for (auto* b : gfech::g_all) b->drop_waits(lane, src);
}
