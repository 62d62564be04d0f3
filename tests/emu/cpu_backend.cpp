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
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_1806_04211_amd/csrc/backend.h"

namespace gfech {
namespace {

class CpuBackend final : public Backend {
public:
    const char* name() const override { return "cpu-emulator"; }
    void* alloc(size_t bytes) override { return calloc(bytes ? bytes : 1, 1); }
    void release(void* p) override { free(p); }
    void zero(void* p, size_t bytes) override { if (bytes) memset(p, 0, bytes); }
    void upload(void* dst, const void* src, size_t bytes) override { if (bytes) memcpy(dst, src, bytes); }
    void download(void* dst, const void* src, size_t bytes) override { if (bytes) memcpy(dst, src, bytes); }
    void copy(void* dst, const void* src, size_t bytes) override { if (bytes) memmove(dst, src, bytes); }
    void sync() override {}

    void gemm(const std::vector<GemmDesc>& ds) override {
        for (const GemmDesc& g : ds) {
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
        for (const GatherDesc& g : ds) {
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
        for (const FillDesc& f : ds) {
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
        for (const ListDesc& l : ds) {
            for (int t = 0; t < l.npick; ++t) l.append[t] = l.add + l.map[l.pick ? l.pick[t] : t];
            for (int s = 0; s < l.nkeep; ++s) l.keep_out[s] = l.map[l.keep ? l.keep[s] : s];
        }
    }

    void sort(const std::vector<SortDesc>& ds) override {
        for (const SortDesc& s : ds) {
            for (int t = 0; t < s.n; ++t) {
                int rank = 0;
                for (int u = 0; u < s.n; ++u) rank += s.vals[u] < s.vals[t];
                s.out[rank] = s.add + (s.mode ? t : s.vals[t]);
            }
        }
    }

    int64_t count_out_of_range(const uint8_t* A, int64_t m, int64_t n, int64_t lda, int32_t p) override {
        int64_t bad = 0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) bad += A[i * lda + j] >= p;
        return bad;
    }

    void ech(const std::vector<EchDesc>& ds) override {
        for (const EchDesc& e : ds) ech_one(e);
    }

private:
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

}  // namespace

Backend* backend_instance(std::string* err) {
    (void)err;
    static CpuBackend be;
    return &be;
}

}  // namespace gfech
