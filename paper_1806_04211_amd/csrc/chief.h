// The Chief (Section 3): the plan of ClearDown / Extend / UpdateRow /
// UpdateRowTrafo tasks (Step 1), RowLengthen (Step 2) and PreClearUp / Copy /
// ClearUp (Step 3) over a block grid, executed layer by layer (layer = i + j,
// Section 5) as grouped launches on a Backend.
#pragma once
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "backend.h"

namespace gfech {

// Algorithmic multiply-adds per task kind, using the cost model of Section 5
// (a product (x by y)(y by z) costs xyz, echelonising x by y of rank r costs xyr).
struct Stats {
    double cd_mad = 0;     // ClearDown's two MADs
    double ech = 0;        // ECH jobs
    double ur_mad = 0;     // UpdateRow MADs / MULs on the data blocks
    double urt_mad = 0;    // UpdateRowTrafo MADs / MULs on the transformation blocks
    double cu_mad = 0;     // ClearUp MADs (Step 3)
    double gather_bytes = 0;   // bytes moved by extracts / riffles / copies
    double mad_bytes = 0;      // operand bytes of the MAD launches: A, B, C read once, D written once
    int64_t layers = 0, echs = 0, gemms = 0, launches = 0, syncs = 0;
    // ClearDowns whose ECH of the leading columns left rows unselected: those
    // whose remnant after them was zero (no second ECH), and those whose ECH
    // ran again on the whole block
    int64_t tail_checks = 0, ech_reruns = 0;
    // kernel time by kind when profiling was requested (device events): gemm, ech, small jobs
    double kernel_ms[3] = {0, 0, 0};
    int64_t kernel_launches[3] = {0, 0, 0};
    double kernel_mac[3] = {0, 0, 0};   // multiply-adds of the timed MAD launches
    double total_mac() const { return cd_mad + ech + ur_mad + urt_mad + cu_mad; }
};

// What a problem computes (the variants of Section 1): everything (the
// reduced echelon form and the transformation), the reduced echelon form
// alone (no UpdateRowTrafo products, no M part of Step 3: M and K are not
// formed), or the rank with the pivot columns and selected rows (Step 3 is
// not run either: R is not reduced and not kept).
enum Want : int32_t { kWantAll = 0, kWantRref = 1, kWantRank = 2 };

// Device-resident result (library-owned).
struct Result {
    Backend* be = nullptr;
    int64_t m = 0, n = 0, r = 0;
    int32_t p = 0;
    int32_t want = kWantAll;         // which outputs were computed (Want)
    // Pfinal: r rows, leading dimension ldP.  Columns [0, r) are scratch (the
    // cleared X blocks), [offR, offR + n - r) hold the remnant R (Eq. (3), rows
    // ordered by pivot column, columns = non-pivot columns ascending),
    // [offM, offM + r) hold M (columns ordered by selected row); offR and offM
    // are the first multiples of 16 at or after r and offR + n - r, so the
    // products of Step 3 see 16-byte aligned rows; the gaps are zero.
    // Without the transformation (kWantRref) there are no M columns (offM is
    // the end of R) and Kfinal holds nothing; for kWantRank Pfinal holds
    // nothing either.
    uint8_t* Pfinal = nullptr; int64_t ldP = 0;
    int64_t offR = 0, offM = 0;
    uint8_t* Kfinal = nullptr; int64_t ldK = 0;   // (m - r) x r
    int32_t* upsilon = nullptr;      // r pivot columns, ascending
    int32_t* upsilon_bar = nullptr;  // n - r
    int32_t* varrho = nullptr;       // r selected rows, ascending
    int32_t* varrho_bar = nullptr;   // m - r
    void* block = nullptr;           // the one allocation all of the above are carved from
    std::vector<void*> pieces;       // or separate allocations (bounds-checking test builds)
    Stats stats;
    std::vector<int32_t> row_blocks, col_blocks;
    ~Result();
};

struct Problem {
    const uint8_t* A = nullptr;   // backend address of the m x n input
    int64_t m = 0, n = 0, lda = 0;
    // or (p = 2) GF(2) rows packed in 64-bit words, ldw words per row, unpacked
    // straight into the block-row panels (no byte copy of the input is made)
    const uint64_t* packed = nullptr;
    int64_t ldw = 0;
    int32_t p = 0;
    int32_t want = kWantAll;
    std::vector<int32_t> row_blocks, col_blocks;   // a_i and b_j (sums m and n)
};

// Choose block sizes (Section 3.1).  A target that is a multiple of 64 gives
// blocks of exactly that size and a smaller last block (the paper notes the
// first and last blocks may be smaller); other targets split evenly.
// target <= 0 means a single block.
std::vector<int32_t> even_blocks(int64_t total, int64_t target);

// The method on any number of independent problems that may join at any
// time.  Each problem is a state machine (Step 1 layer by layer, then the
// assembly of the result and Step 2, then Step 3's ClearUp launches one per
// iteration); one call of step() advances every active problem by one phase,
// and the jobs of all problems in the same phase share launches.  Problems
// added between calls of step() join the next iteration (continuous batching).
class Engine {
public:
    explicit Engine(Backend& be);
    ~Engine();
    // Device bytes a problem holds while active (its block arena, the result,
    // the assembly maps), an upper bound.
    size_t footprint(const Problem& pr) const;
    // Adds a problem (copied; its input must stay valid until it finishes).
    // Returns its id (>= 0), or -1 with *status set (device memory exhausted).
    int64_t add(const Problem& pr, int* status);
    // One iteration; returns the number of problems still active.
    size_t step();
    // Stops problem `id` at the next iteration: its queued work completes,
    // its memory is freed and it finishes with status kCancelled (no result).
    void cancel(int64_t id);
    size_t active() const;
    size_t bytes_in_use() const;
    // Problems finished since the last call: id, status (0 or a backend error
    // code) and the result (null on error).
    struct Done {
        int64_t id = -1;
        int status = 0;
        std::unique_ptr<Result> result;
    };
    std::vector<Done> take_done();
    // launches, gemms, syncs and layers of every iteration so far
    const Stats& totals() const;

private:
    struct Impl;
    std::unique_ptr<Impl> impl_;
};

// Status of a problem stopped by Engine::cancel (or the watchdog of run_chief).
constexpr int kCancelled = 7;

// Run the whole method on a set of independent problems in lockstep (their
// jobs share launches).  Returns 0 or a backend error code; results are
// appended to `out` in problem order.  timeout_ms > 0 is a watchdog: problems
// still running after that long are cancelled and the call returns kCancelled.
int run_chief(Backend& be, const std::vector<Problem>& probs,
              std::vector<std::unique_ptr<Result>>& out, std::string* err, int profile = 0,
              int64_t timeout_ms = 0);

}  // namespace gfech
