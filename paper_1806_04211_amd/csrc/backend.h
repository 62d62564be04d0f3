// Job-level interface between the host planner (the Chief) and the device.
//
// Every operation is *grouped*: the planner hands over all independent jobs of
// one phase at once and the backend runs them in a single launch.  Pointers in
// the descriptors are addresses in the backend's memory (HBM for the HIP
// backend).  Shapes are exact; the planner never asks a backend to touch
// bytes outside the extents a descriptor states.
#pragma once
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <vector>

namespace gfech {

// MAD / MUL job (Section 4.1): D = (Cin + A * B) mod p.
//   A   : M x K, row-major, leading dimension lda
//   B   : K x N; row t of B is row brow[t] of the base when brow != nullptr
//   Cin : M x N; nullptr means zero; row x is row crow[x] of the base when crow != nullptr
//   D   : M x N output.  D may equal Cin when crow == nullptr and ldc == ldd
//         (element-wise in place); D never overlaps A or B.
// Entries are canonical residues in [0, p); K may be 0 (then D = Cin).
constexpr int32_t kGemmRowsPadded = 1;
enum GemmKind : int32_t { kGemmOther = 0, kGemmClearDown = 1, kGemmUpdateRow = 2, kGemmUpdateRowTrafo = 3,
                          kGemmClearUp = 4 };

struct GemmDesc {
    int32_t M = 0, N = 0, K = 0, p = 0;
    // kGemmRowsPadded: every row of B and C may be read up to the next
    // multiple of 16 columns past N (the buffers hold whole rows of their
    // leading dimension); set by the planner for its own buffers
    int32_t flags = 0;
    int32_t kind = 0;   // what the product is for (GemmKind), for traces only

    const uint8_t* A = nullptr; int64_t lda = 0;
    const uint8_t* B = nullptr; int64_t ldb = 0; const int32_t* brow = nullptr;
    const uint8_t* C = nullptr; int64_t ldc = 0; const int32_t* crow = nullptr;
    uint8_t* D = nullptr; int64_t ldd = 0;
};

// Permuted copy (the extract / riffle jobs CEX, REX, RRF of Section 4.1):
//   dst[drow[x]][dcol[y]] = f(src[srow[x]][scol[y]])   for x < rows, y < cols
// with each map optional (identity when nullptr) and f(v) = v, or
// f(v) = (neg_p - v) mod neg_p when neg_p != 0 (negation in GF(neg_p)).
struct GatherDesc {
    int32_t rows = 0, cols = 0, neg_p = 0;
    const uint8_t* src = nullptr; int64_t lds = 0;
    const int32_t* srow = nullptr; const int32_t* scol = nullptr;
    uint8_t* dst = nullptr; int64_t ldd = 0;
    const int32_t* drow = nullptr; const int32_t* dcol = nullptr;
};

// Fill dst (rows x cols) with `value`; when diag_value >= 0 the entries
// (t, t) are set to diag_value instead (identity-like fills).  When dcol is
// given only the entries (t, dcol[t]), t < rows, are written, with diag_value
// (a scattered identity); `cols` is then unused.
struct FillDesc {
    int32_t rows = 0, cols = 0;
    uint8_t* dst = nullptr; int64_t ldd = 0;
    int32_t value = 0, diag_value = -1;
    const int32_t* dcol = nullptr;
};

// ECH job (Remark 2.3) on H (rows x cols).  With r = rank(H), outputs
//   rcount[0] = r
//   prow[t]   (t < r)        : row of the t-th pivot, pivots ordered by column
//   qrow[s]   (s < rows-r)   : non-pivot rows, ascending
//   pcol[t]   (t < r)        : pivot columns, ascending
//   qcol[s]   (s < cols-r)   : non-pivot columns, ascending
//   Mo (r x r), Ko ((rows-r) x r), Ro (r x (cols-r)) with
//   [[Mo,0],[Ko,1]] [H[prow]; H[qrow]] [H cols pcol | qcol] = [[-1, Ro],[0,0]].
// Pivot rule of the paper: a column's pivot is the first not-yet-selected row
// (in H's row order) that is non-zero there after elimination.  `work` is
// scratch of rows x (cols + min(rows, cols)) bytes with leading dimension ldw.
struct EchDesc {
    int32_t rows = 0, cols = 0, p = 0;
    // qcol continues with cols, cols + 1, .., cols + qtail - 1 (columns of the
    // caller's beyond the ones given, known to hold no pivot)
    int32_t qtail = 0;
    const uint8_t* H = nullptr; int64_t ldh = 0;
    uint8_t* work = nullptr; int64_t ldw = 0;
    int32_t* rcount = nullptr;
    int32_t* prow = nullptr; int32_t* qrow = nullptr;
    int32_t* pcol = nullptr; int32_t* qcol = nullptr;
    uint8_t* Mo = nullptr; int64_t ldm = 0;
    uint8_t* Ko = nullptr; int64_t ldk = 0;
    uint8_t* Ro = nullptr; int64_t ldr = 0;
};

// Index-list update used by Extend / UNH (Section 4.2) and ClearDown's UNH:
//   append[t]  = add + map[pick[t]]   for t < npick   (new elements, in pick order)
//   keep_out[s] = map[keep[s]]        for s < nkeep   (the remaining complement)
// A null pick or keep means the identity (t, s); a null map means the
// identity too (so map == pick == nullptr writes add + t).
// keep_out must not alias map.
struct ListDesc {
    int32_t npick = 0, nkeep = 0, add = 0;
    const int32_t* map = nullptr;
    const int32_t* pick = nullptr; int32_t* append = nullptr;
    const int32_t* keep = nullptr; int32_t* keep_out = nullptr;
};

// MAD over GF(2) on bit-packed rows (bit b of 64-bit word w = column 64 w + b):
//   D = C + A * B   (XOR of the rows of B selected by the bits of each row of A)
//   A: M x K bits, lda words per row (its bits past K - 1 are ignored)
//   B: K x N bits, ldb words; C (or nullptr = zero) and D: M x N bits, ldc / ldd
//   words.  Bits of B and C past column N - 1 must be zero (D's then are).
//   D may equal C (same ld); D never overlaps A or B.
struct Gf2MadDesc {
    int64_t M = 0, N = 0, K = 0;
    const uint64_t* A = nullptr; int64_t lda = 0;
    const uint64_t* B = nullptr; int64_t ldb = 0;
    const uint64_t* C = nullptr; int64_t ldc = 0;
    uint64_t* D = nullptr; int64_t ldd = 0;
};

// Sorting of small distinct-valued lists (for the final row and column orders):
//   mode 0: out[k] = add + (k-th smallest value)
//   mode 1: out[k] = add + (index of the k-th smallest value)
struct SortDesc {
    int32_t n = 0, mode = 0, add = 0;
    const int32_t* vals = nullptr;
    int32_t* out = nullptr;
};

// Size of the fixed device workspace (one per device, held until the process
// ends) that the allocation-free ECH entry point uses instead of an allocation.
constexpr size_t kFixedScratchBytes = (size_t)16 << 20;

class Backend {
public:
    virtual ~Backend() = default;
    // Every use of an instance is serialised by its lock (its stream, lanes,
    // marks and memory cache are per instance).
    std::mutex& lock() { return mu_; }
    virtual const char* name() const = 0;
    // memory (alloc does not initialise; nullptr on failure)
    virtual void* alloc(size_t bytes) = 0;
    virtual void release(void* ptr) = 0;
    virtual void zero(void* ptr, size_t bytes) = 0;
    virtual void upload(void* dst, const void* host_src, size_t bytes) = 0;
    virtual void download(void* host_dst, const void* src, size_t bytes) = 0;   // waits for prior work
    virtual void copy(void* dst, const void* src, size_t bytes) = 0;            // device to device
    // grouped jobs, executed in submission order
    virtual void gemm(const std::vector<GemmDesc>& d) = 0;
    virtual void gather(const std::vector<GatherDesc>& d) = 0;
    virtual void fill(const std::vector<FillDesc>& d) = 0;
    virtual void ech(const std::vector<EchDesc>& d) = 0;
    virtual void lists(const std::vector<ListDesc>& d) = 0;
    virtual void sort(const std::vector<SortDesc>& d) = 0;
    virtual void sync() = 0;
    // waits for lane 0's work only (the other lanes may still run)
    virtual void sync_lane0() { sync(); }
    // number of entries >= p in an m x n matrix (waits for the answer)
    virtual int64_t count_out_of_range(const uint8_t* A, int64_t m, int64_t n, int64_t lda, int32_t p) = 0;
    // the same for many matrices at once, one answer per matrix (one wait in all)
    struct RangeDesc {
        const uint8_t* A = nullptr;
        int64_t m = 0, n = 0, lda = 0;
        int32_t p = 0;
    };
    virtual void count_out_of_range_many(const std::vector<RangeDesc>& ds, std::vector<int64_t>& bad) {
        bad.assign(ds.size(), 0);
        for (size_t t = 0; t < ds.size(); ++t) bad[t] = count_out_of_range(ds[t].A, ds[t].m, ds[t].n, ds[t].lda, ds[t].p);
    }
    // GF(2) rows packed in 64-bit words, bit b of word w = column 64 w + b, to
    // one byte per entry: dst[x][y] = bit (y mod 64) of src[x][y / 64] for
    // x < m, y < n (ldw words and ldd bytes per row)
    virtual void unpack_gf2(const uint64_t* src, int64_t m, int64_t n, int64_t ldw, uint8_t* dst, int64_t ldd) = 0;
    // one MAD over GF(2) on packed rows (ordered on the current lane)
    virtual void mad_gf2(const Gf2MadDesc& d) = 0;
    // number of rows whose last word has a set bit past column n - 1 (waits for the answer)
    virtual int64_t count_gf2_pad(const uint64_t* src, int64_t m, int64_t n, int64_t ldw) = 0;
    // stream for subsequent work (a hipStream_t for the HIP backend)
    virtual void set_stream(void* stream) { (void)stream; }
    // a stream of the library's own (default priority), and its release
    virtual void* create_stream() { return nullptr; }
    virtual void destroy_stream(void* stream) { (void)stream; }
    // Four lanes of work: lane 0 is the caller's stream, lanes 1, 2 and 3
    // streams whose work may overlap lane 0's and each other's.  mark() records the
    // point reached by a lane's queued work; wait_mark() makes a lane wait for
    // such a point (of any lane).  Memory transfers (upload, download, zero,
    // copy) always run on lane 0.
    virtual void set_lane(int lane) { (void)lane; }
    virtual int mark(int lane) { (void)lane; return 0; }
    virtual void wait_mark(int lane, int mark) { (void)lane; (void)mark; }
    // A small int32 array that jobs write on the device and read_counts()
    // returns to the host once lane 0's queued work is complete (lane 1 may
    // still be running).  One array per backend, valid until the next call.
    virtual int32_t* counts_buffer(size_t n) { return (int32_t*)alloc(sizeof(int32_t) * n); }
    virtual void read_counts(int32_t* host, const int32_t* counts, size_t n) {
        download(host, counts, sizeof(int32_t) * n);
    }
    virtual void release_counts(int32_t* counts) { release(counts); }
    // The fixed workspace of kFixedScratchBytes (nullptr when unavailable):
    // device memory that is never allocated or freed after initialisation.
    virtual uint8_t* fixed_scratch() { return nullptr; }
    // non-zero after a device error; the planner stops and reports it
    virtual int error() const { return 0; }
    // per-launch timing of the grouped jobs (device events on the work stream)
    struct Profile {
        double ms[4] = {0, 0, 0, 0};        // gemm, ech, gather/fill/lists/sort, range check
        int64_t launches[4] = {0, 0, 0, 0};
        double mac[4] = {0, 0, 0, 0};       // multiply-adds of the timed MAD launches
    };
    virtual void set_profile(int level) { (void)level; }   // 0 off, 1 every launch, 2 MAD launches only
    virtual Profile take_profile() { return Profile(); }

private:
    std::mutex mu_;
};

}  // namespace gfech
