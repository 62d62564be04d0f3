// The Chief (Section 3, "The Chief"): Step 1 (ClearDown, Extend, UpdateRow,
// UpdateRowTrafo), Step 2 (RowLengthen) and Step 3 (PreClearUp, Copy,
// ClearUp), executed layer by layer (layer i + j, Section 5) as grouped jobs.
//
// Storage differs from the paper's in one respect, chosen for the GPU: the
// pivot rows of a block column, the pivot columns of D.gamma and the selected
// rows of a block row are kept in the order they were found ("append order")
// instead of sorted order.  The riffles then become appends: RRF with
// lambda = (0..0 1..1), CRZ = extend with zero columns at the end, ADI =
// identity columns at the end, RowLengthen = nothing to do.  One permutation
// when the result is assembled restores the sorted orders of Eq. (2).  Every
// product the paper computes is computed on the same operands, merely with
// rows / columns stored in another order.
//
// Block-row data are held as panels: block row i's blocks C_i,k for k > j are
// one a_i x n panel (so UpdateRow(i, j, k) for all k > j is one MAD), and its
// transformation blocks K_i,h (h <= i) sit side by side in one panel, each in
// a column range reserved for block row h.  The pivot rows B_j,k and M_j,h of
// block column j live in rows of one pivot matrix P.
//
// Lookahead on four lanes (streams).  Every UpdateRow / UpdateRowTrafo
// product is column-separable: output column c depends only on column c of
// its inputs.  So the products of task (i, j) are split by output columns
// into a priority part, block column j + 1 (the one the next ClearDown of
// block row i reads), and a bulk part: a near set (block column j + 2, which
// the next layer's priority part of block row i overwrites), a mid set
// (block column j + 3, the next layer's near set) and a far set (block
// columns j + 4.. and every transformation column).  Lane 0 runs the
// ClearDowns and the priority part; lane 1 runs the previous layer's near
// and mid sets, lane 3 its far set, both starting after the ClearDown MADs
// and issued after the ECHs so that the ECHs reach the device first; lane 2
// runs the priority part of UpdateRow (1), which needs the near set and
// nothing the ECH computes, beside the ECH.  Lane 0 waits for lane 2 (so for
// the near set) before the rest of the layer's products.  The sets of
// consecutive layers of a block row update the same blocks from block
// column j + 3 on, so a mid set waits for the previous layer's far set
// (block j + 3 is in both); the far sets follow each other on lane 3 and run
// beside the next layer's near set.  The job scratch the bulk part reads
// (A.A, A.M, A.K, A.E, the row lists of the ECH) is kept in three copies, by
// layer mod 3; lane 0 waits for a far set before the ClearDowns of the
// layer that reuses its copy.
#include "chief.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

namespace gfech {

Result::~Result() {
    if (!be) return;
    be->release(block);
    for (void* v : pieces) be->release(v);
}

std::vector<int32_t> even_blocks(int64_t total, int64_t target) {
    std::vector<int32_t> v;
    if (total <= 0) return v;
    if (target <= 0 || target >= total) {
        v.push_back((int32_t)total);
        return v;
    }
    // targets that are multiples of 64 give blocks of exactly `target` (aligned
    // panels for the vector loads) and a smaller last block; other targets are
    // split evenly
    if (target % 64 == 0) {
        for (int64_t off = 0; off < total; off += target) v.push_back((int32_t)std::min<int64_t>(target, total - off));
        return v;
    }
    int64_t k = (total + target - 1) / target;
    for (int64_t i = 0; i < k; ++i) v.push_back((int32_t)(total / k + (i < total % k ? 1 : 0)));
    return v;
}

namespace {

constexpr size_t kAlign = 256;

struct Arena {
    size_t size = 0;
    std::vector<std::pair<size_t, size_t>> slots;   // (offset, bytes) of every sub-buffer
    size_t take(size_t bytes) {
        size_t off = size;
        slots.push_back({off, bytes});
        size += (bytes + kAlign - 1) / kAlign * kAlign;
        return off;
    }
};

struct Ops {
    std::vector<GemmDesc> gemm;
    std::vector<GatherDesc> gather;
    std::vector<ListDesc> lists;
    std::vector<EchDesc> ech;
    std::vector<SortDesc> sort;
    std::vector<FillDesc> fill;
    bool empty() const {
        return gemm.empty() && gather.empty() && lists.empty() && ech.empty() && sort.empty() && fill.empty();
    }
};

// The bulk part of a layer's UpdateRow / UpdateRowTrafo products: `near` holds
// the columns of the block column after the priority one (which the next
// layer's priority products of the same block row overwrite), `mid` those of
// the block column after that (the next layer's near set), `far` the rest.
struct Bulk {
    Ops near, mid, far;
    bool empty() const { return near.empty() && mid.empty() && far.empty(); }
};

// Copies of the per-block-column job scratch, used round robin by layer: the
// bulk part of layer L reads copy L mod kScratchCopies while layers L + 1 and
// L + 2 write the other copies
constexpr int kScratchCopies = 3;
// regions up to this size are zeroed by the fill job (one launch for all of
// them), larger ones by a memset
constexpr int64_t kFillZeroMax = 4 << 20;

struct TaskState {      // one (i, j) of the current layer
    int i = 0, j = 0;
    int par = 0;        // which copy of the job scratch this layer uses (layer mod kScratchCopies)
    bool active = false, did_ech = false;
    int32_t alpha = 0;  // rows of block row i when the layer started
    int32_t r = 0;      // pivots of block column j before ClearDown
    int32_t rp = 0;     // new pivots r'
    // ECH of the leading columns only (see cd_ech)
    int32_t w = 0;      // columns the ECH was given
    bool split = false; // w < all columns of H
    bool rerun = false; // the leading columns did not select every row: ECH again on all of H
    const uint8_t* H = nullptr;
    int64_t ldh = 0;
};

// Columns beyond the number of rows the leading-columns ECH is given
constexpr int32_t kSplitSlack = 32;

class Plan {
public:
    Plan(Backend& be, const Problem& pr, Stats& st) : be_(be), pr_(pr), st_(st) {
        a_ = (int)pr.row_blocks.size();
        b_ = (int)pr.col_blocks.size();
        m_ = pr.m;
        n_ = pr.n;
        p_ = pr.p;
        R0_.assign(a_ + 1, 0);
        C0_.assign(b_ + 1, 0);
        for (int i = 0; i < a_; ++i) R0_[i + 1] = R0_[i] + pr.row_blocks[i];
        for (int j = 0; j < b_; ++j) C0_[j + 1] = C0_[j] + pr.col_blocks[j];
        alpha_.assign(pr.row_blocks.begin(), pr.row_blocks.end());
        rankc_.assign(b_, 0);
        sel_.assign(a_, std::vector<int32_t>(b_, 0));
        trafo_ = pr.want == kWantAll;
        keepR_ = pr.want != kWantRank;
        amax_ = a_ ? *std::max_element(pr.row_blocks.begin(), pr.row_blocks.end()) : 0;
    }

    int layers() const { return (a_ && b_) ? a_ + b_ - 1 : 0; }
    int blockcols() const { return b_; }

    // ------------------------------------------------------------ memory
    // Two arenas: the block-row panels C (needed in Step 1 only, so freed
    // before the result is assembled) and everything else.  plan_memory
    // returns the total; panel_bytes() the panels' part.
    size_t plan_memory() {
        Arena ar, arc;
        rows_.resize(a_);
        cols_.resize(b_);
        for (int i = 0; i < a_; ++i) {
            BR& br = rows_[i];
            int64_t ai = pr_.row_blocks[i];
            // 64-byte aligned rows, so the products take the streamed MAD path
            br.ldC = std::max<int64_t>((n_ + 63) / 64 * 64, 64);
            br.ldK = trafo_ ? (R0_[i] + ai + 63) / 64 * 64 : 0;
            for (int s = 0; s < 2; ++s) {
                br.oC[s] = arc.take(ai * br.ldC);
                br.oK[s] = ar.take(ai * br.ldK);
                br.oU[s] = ar.take(sizeof(int32_t) * ai);
            }
            br.oE = ar.take(sizeof(int32_t) * ai);
        }
        int64_t prow = 0;
        for (int j = 0; j < b_; ++j) {
            BC& bc = cols_[j];
            int64_t bj = pr_.col_blocks[j];
            bc.cap = std::min<int64_t>(bj, m_);
            bc.ld = bj;
            bc.prow0 = prow;
            prow += bc.cap;
            for (int s = 0; s < 2; ++s) {
                bc.oDR[s] = ar.take(bc.cap * bj);
                bc.oGbar[s] = ar.take(sizeof(int32_t) * bj);
            }
            bc.oGam = ar.take(sizeof(int32_t) * bj);
            for (int s = 0; s < kScratchCopies; ++s) {
                bc.oAA[s] = ar.take(amax_ * bj);
                bc.oAM[s] = ar.take(bj * bj);
                bc.oAK[s] = ar.take(amax_ * bj);
                bc.oProw[s] = ar.take(sizeof(int32_t) * std::max<int64_t>(amax_, 1));
                bc.oQrow[s] = ar.take(sizeof(int32_t) * std::max<int64_t>(amax_, 1));
                bc.oAE[s] = ar.take(bc.cap * bj);
            }
            bc.oH = ar.take(amax_ * bj);
            bc.ldW = 2 * bj;
            bc.oW = ar.take(amax_ * bc.ldW);
            bc.oPcol = ar.take(sizeof(int32_t) * bj);
            bc.oQcol = ar.take(sizeof(int32_t) * bj);
        }
        prow_total_ = prow;
        // pivot rows: n data columns, then (with the transformation) m columns of M
        ldP_ = std::max<int64_t>((n_ + (trafo_ ? m_ : 0) + 63) / 64 * 64, 64);
        oP_ = ar.take(prow_total_ * ldP_);
        arena_bytes_ = ar.size;
        panel_bytes_ = arc.size;
        slots_ = ar.slots;
        panel_slots_ = arc.slots;
        return ar.size + arc.size;
    }
    size_t panel_bytes() const { return panel_bytes_; }

    const std::vector<std::pair<size_t, size_t>>& slots() const { return slots_; }
    const std::vector<std::pair<size_t, size_t>>& panel_slots() const { return panel_slots_; }

    // at(offset) gives the address of the sub-buffer planned at that offset of
    // the main arena, atc(offset) of the panels' arena
    template <typename At, typename AtC>
    void bind(At at, AtC atc, int32_t* counts) {
        counts_ = counts;
        for (auto& br : rows_) {
            for (int s = 0; s < 2; ++s) {
                br.C[s] = atc(br.oC[s]);
                br.K[s] = at(br.oK[s]);
                br.U[s] = (int32_t*)at(br.oU[s]);
            }
            br.E = (int32_t*)at(br.oE);
        }
        for (auto& bc : cols_) {
            for (int s = 0; s < 2; ++s) {
                bc.DR[s] = at(bc.oDR[s]);
                bc.Gbar[s] = (int32_t*)at(bc.oGbar[s]);
            }
            for (int s = 0; s < kScratchCopies; ++s) {
                bc.AA[s] = at(bc.oAA[s]);
                bc.AM[s] = at(bc.oAM[s]);
                bc.AK[s] = at(bc.oAK[s]);
                bc.Prow[s] = (int32_t*)at(bc.oProw[s]);
                bc.Qrow[s] = (int32_t*)at(bc.oQrow[s]);
                bc.AE[s] = at(bc.oAE[s]);
            }
            bc.Gam = (int32_t*)at(bc.oGam);
            bc.H = at(bc.oH);
            bc.W = at(bc.oW);
            bc.Pcol = (int32_t*)at(bc.oPcol);
            bc.Qcol = (int32_t*)at(bc.oQcol);
        }
        P_ = at(oP_);
    }

    // zero what must start at zero, load the input, initialise the index lists.
    // Small regions are zeroed by the fill job, which takes every region of a
    // batch in one launch (a memset costs the host a few microseconds each:
    // three per matrix made a third of a batch of 4096 small matrices).
    void init(Ops& ops) {
        const auto zero = [&](uint8_t* p, int64_t rows, int64_t ld) {
            if (rows <= 0 || ld <= 0) return;
            if (rows * ld <= kFillZeroMax) {
                FillDesc f;
                f.rows = (int32_t)rows;
                f.cols = (int32_t)ld;
                f.dst = p;
                f.ldd = ld;
                ops.fill.push_back(f);
            } else {
                be_.zero(p, (size_t)(rows * ld));
            }
        };
        zero(P_, prow_total_, ldP_);
        for (int i = 0; i < a_; ++i) {
            BR& br = rows_[i];
            int64_t ai = pr_.row_blocks[i];
            if (trafo_) {
                zero(br.K[0], ai, br.ldK);
                zero(br.K[1], ai, br.ldK);
            }
            if (n_ > 0 && pr_.packed) {
                // GF(2) packed rows straight into the panel (a lane-0 job)
                be_.unpack_gf2(pr_.packed + R0_[i] * pr_.ldw, ai, n_, pr_.ldw, br.C[0], br.ldC);
            } else if (n_ > 0) {
                GatherDesc g;
                g.rows = (int32_t)ai;
                g.cols = (int32_t)n_;
                g.src = pr_.A + R0_[i] * pr_.lda;
                g.lds = pr_.lda;
                g.dst = br.C[0];
                g.ldd = br.ldC;
                ops.gather.push_back(g);
            }
            ListDesc l;                       // U = 0 .. a_i - 1
            l.npick = (int32_t)ai;
            l.append = br.U[0];
            ops.lists.push_back(l);
        }
        for (int j = 0; j < b_; ++j) {
            ListDesc l;                       // Gamma-bar = 0 .. b_j - 1
            l.npick = pr_.col_blocks[j];
            l.append = cols_[j].Gbar[0];
            ops.lists.push_back(l);
        }
    }

    // ------------------------------------------------------------ Step 1, one layer
    void begin_layer(int L) {
        tasks_.clear();
        int ilo = std::max(0, L - b_ + 1), ihi = std::min(a_ - 1, L);
        for (int i = ilo; i <= ihi; ++i) {
            TaskState t;
            t.i = i;
            t.j = L - i;
            t.alpha = alpha_[i];
            t.r = rankc_[t.j];
            t.par = L % kScratchCopies;
            t.active = t.alpha > 0;
            tasks_.push_back(t);
        }
    }

    // ClearDown: CEX of C by D.gamma (A.A and A')
    void cd_extract(Ops& ops) {
        for (auto& t : tasks_) {
            if (!t.active) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            const uint8_t* Cij = br.C[br.cur] + C0_[t.j];
            if (t.r > 0) {
                GatherDesc g;
                g.rows = t.alpha; g.cols = t.r;
                g.src = Cij; g.lds = br.ldC; g.scol = bc.Gam;
                g.dst = bc.AA[t.par]; g.ldd = bj;
                ops.gather.push_back(g);
                st_.gather_bytes += 2.0 * t.alpha * t.r;
                if (bj - t.r > 0) {
                    GatherDesc h = g;
                    h.cols = bj - t.r; h.scol = bc.Gbar[bc.gcur];
                    h.dst = bc.H;
                    ops.gather.push_back(h);
                    st_.gather_bytes += 2.0 * t.alpha * (bj - t.r);
                }
            }
        }
    }

    // ClearDown's first MAD: H = A' + A.A * D.R
    void cd_mad(Ops& ops) {
        for (auto& t : tasks_) {
            if (!t.active || t.r == 0) continue;
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            if (bj - t.r == 0) continue;
            GemmDesc g;
            g.M = t.alpha; g.N = bj - t.r; g.K = t.r; g.p = p_;
            g.A = bc.AA[t.par]; g.lda = bj;
            g.B = bc.DR[bc.dcur]; g.ldb = bc.ld;
            g.C = bc.H; g.ldc = bj; g.D = bc.H; g.ldd = bj;
            push_gemm(ops, g, st_.cd_mad);
        }
    }

    // UpdateRow / UpdateRowTrafo step (1): Z := C + A.A * B over all blocks
    // k > j of the panel, and Z := K + A.A * M for h != i (K's new columns are
    // the zero columns CRZ adds)
    void ur1(Ops& pri, Bulk& bulk) {
        for (auto& t : tasks_) {
            if (!t.active || t.r == 0) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            int64_t c0 = C0_[t.j + 1];
            if (n_ - c0 > 0) {
                GemmDesc g;
                g.M = t.alpha; g.N = (int32_t)(n_ - c0); g.K = t.r; g.p = p_;
                g.A = bc.AA[t.par]; g.lda = bj;
                g.B = P_ + bc.prow0 * ldP_ + c0; g.ldb = ldP_;
                g.C = br.C[br.cur] + c0; g.ldc = br.ldC;
                g.D = br.C[br.cur] + c0; g.ldd = br.ldC;
                push_split(pri, bulk, g, t.j, st_.ur_mad);
            }
            for (int h = 0; trafo_ && h < t.i; ++h) {
                int32_t w = sel_[h][t.j];
                if (w == 0) continue;
                GemmDesc g;
                g.M = t.alpha; g.N = w; g.K = t.r; g.p = p_;
                g.A = bc.AA[t.par]; g.lda = bj;
                g.B = P_ + bc.prow0 * ldP_ + n_ + R0_[h]; g.ldb = ldP_;
                g.C = br.K[br.cur] + R0_[h]; g.ldc = br.ldK;
                g.D = br.K[br.cur] + R0_[h]; g.ldd = br.ldK;
                push_gemm(bulk.far, g, st_.urt_mad);
            }
        }
    }

    // ClearDown's ECH.  When H has more than alpha + kSplitSlack columns, the
    // ECH first gets only the leading alpha + kSplitSlack of them.  If that
    // selects every row (the usual case for a block of full row rank), no
    // later column can hold a pivot, and the remnant of the remaining columns
    // H2 is R2 = M H2[rho'] (the top rows of the identity of Remark 2.3), one
    // product on the whole device instead of a trailing update inside the ECH
    // (cd_post).  Otherwise the ECH runs again on all of H (rerun pass).
    void cd_ech(Ops& ops, bool rerun_pass) {
        for (auto& t : tasks_) {
            if (!t.active) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            const int32_t w = bj - t.r;
            if (w == 0) continue;
            if (rerun_pass) {
                if (!t.rerun) continue;
                t.w = w;
                t.split = false;
            } else {
                t.w = (w > t.alpha + kSplitSlack) ? t.alpha + kSplitSlack : w;
                t.split = t.w < w;
            }
            if (t.r > 0) { t.H = bc.H; t.ldh = bj; }
            else { t.H = br.C[br.cur] + C0_[t.j]; t.ldh = br.ldC; }
            EchDesc e;
            e.rows = t.alpha; e.cols = t.w; e.p = p_;
            // the columns after the leading ones hold no pivot when every row is
            // selected there (otherwise the ECH runs again on all of H)
            e.qtail = t.split ? w - t.w : 0;
            e.H = t.H; e.ldh = t.ldh;
            e.work = bc.W; e.ldw = bc.ldW;
            e.rcount = counts_ + t.j;
            e.prow = bc.Prow[t.par]; e.qrow = bc.Qrow[t.par]; e.pcol = bc.Pcol; e.qcol = bc.Qcol;
            e.Mo = bc.AM[t.par]; e.ldm = bj;
            e.Ko = bc.AK[t.par]; e.ldk = bj;
            e.Ro = bc.DR[1 - bc.dcur] + (int64_t)t.r * bc.ld; e.ldr = bc.ld;
            ops.ech.push_back(e);
            t.did_ech = true;
        }
    }

    bool any_ech() const {
        for (auto& t : tasks_) if (t.did_ech) return true;
        return false;
    }

    // returns true when some task needs the rerun pass
    bool absorb_counts(const int32_t* host_counts, bool rerun_pass) {
        bool again = false;
        for (auto& t : tasks_) {
            if (!t.did_ech || (rerun_pass && !t.rerun)) continue;
            t.rp = host_counts[t.j];
            st_.ech += (double)t.alpha * t.w * t.rp;
            if (rerun_pass) {
                t.rerun = false;
                st_.ech_reruns += 1;
            } else {
                st_.echs += 1;
                t.rerun = t.split && t.rp < t.alpha;
                again = again || t.rerun;
            }
        }
        return again;
    }

    void clear_counts() {
        for (auto& t : tasks_) t.rp = 0;
    }

    // A task whose ECH of the leading t.w columns left rows unselected (t.rerun):
    // by the identity of Remark 2.3 on the leading columns, K H[rho'] + H[rho'-bar]
    // vanishes there, and the rows rho'-bar reduced by the pivot rows found are
    // Z = K H[rho', tail] + H[rho'-bar, tail] on the columns after them.  When
    // Z is zero no column after the leading ones holds a pivot (Section 2.3.2's
    // splitting of ech by columns, with an empty second half): the result of the
    // leading columns stands as for a full selection (its K already reduces
    // rho'-bar to zero on every column; the remnant product of cd_post gives R's
    // columns after them), and the ECH need not run again on all of H.  Z goes
    // to the ECH workspace (no ECH reads it now).
    void cd_tail(Ops& ops) {
        for (auto& t : tasks_) {
            if (!t.rerun || t.rp == 0) continue;
            BC& bc = cols_[t.j];
            const int32_t bj = pr_.col_blocks[t.j];
            GemmDesc g;
            g.M = t.alpha - t.rp; g.N = bj - t.r - t.w; g.K = t.rp; g.p = p_;
            g.A = bc.AK[t.par]; g.lda = bj;
            g.B = t.H + t.w; g.ldb = t.ldh; g.brow = bc.Prow[t.par];
            g.C = t.H + t.w; g.ldc = t.ldh; g.crow = bc.Qrow[t.par];
            g.D = bc.W; g.ldd = bc.ldW;
            push_gemm(ops, g, st_.cd_mad);
        }
    }
    // one range check per task of cd_tail (p = 1 counts the non-zero entries of
    // Z; with no pivot among the leading columns Z is the tail of H itself)
    void tail_ranges(std::vector<Backend::RangeDesc>& rd) const {
        for (auto& t : tasks_) {
            if (!t.rerun) continue;
            const BC& bc = cols_[t.j];
            Backend::RangeDesc d;
            if (t.rp > 0) {
                d.A = bc.W; d.m = t.alpha - t.rp; d.lda = bc.ldW;
            } else {
                d.A = t.H + t.w; d.m = t.alpha; d.lda = t.ldh;
            }
            d.n = pr_.col_blocks[t.j] - t.r - t.w;
            d.p = 1;
            rd.push_back(d);
        }
    }
    // the counts in the order of tail_ranges, from nz[pos] on; returns true
    // when some task still needs the ECH on all of H
    bool absorb_tail(const std::vector<int64_t>& nz, size_t& pos) {
        bool again = false;
        for (auto& t : tasks_) {
            if (!t.rerun) continue;
            const int64_t c = pos < nz.size() ? nz[pos] : -1;
            ++pos;
            if (c == 0) {
                t.rerun = false;
                st_.tail_checks += 1;
            } else {
                again = true;
            }
        }
        return again;
    }

    // ClearDown after ECH: CEX of D.R by gamma' (A.E and R'), UNH on D.gamma, Extend on E.rho
    void cd_post(Ops& ops) {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            int32_t rest = bj - t.r - t.rp;
            if (t.split) {
                // every row was selected in the leading t.w columns: the other
                // columns are non-pivot columns, and their remnant is M * H2[rho']
                const int32_t w = bj - t.r;
                GemmDesc g;
                g.M = t.rp; g.N = w - t.w; g.K = t.rp; g.p = p_;
                g.A = bc.AM[t.par]; g.lda = bj;
                g.B = t.H + t.w; g.ldb = t.ldh; g.brow = bc.Prow[t.par];
                g.D = bc.DR[1 - bc.dcur] + (int64_t)t.r * bc.ld + (t.w - t.rp); g.ldd = bc.ld;
                push_gemm(ops, g, st_.cd_mad);
            }
            if (t.r > 0) {
                GatherDesc g;
                g.rows = t.r; g.cols = t.rp;
                g.src = bc.DR[bc.dcur]; g.lds = bc.ld; g.scol = bc.Pcol;
                g.dst = bc.AE[t.par]; g.ldd = bj;
                ops.gather.push_back(g);
                st_.gather_bytes += 2.0 * t.r * t.rp;
                if (rest > 0) {
                    GatherDesc h = g;
                    h.cols = rest; h.scol = bc.Qcol;
                    h.dst = bc.DR[1 - bc.dcur]; h.ldd = bc.ld;
                    ops.gather.push_back(h);
                    st_.gather_bytes += 2.0 * t.r * rest;
                }
            }
            // UNH(D.gamma, gamma'): new pivots appended, complement filtered
            ListDesc lg;
            lg.npick = t.rp; lg.nkeep = rest; lg.map = bc.Gbar[bc.gcur];
            lg.pick = bc.Pcol; lg.append = bc.Gam + t.r;
            lg.keep = bc.Qcol; lg.keep_out = bc.Gbar[1 - bc.gcur];
            ops.lists.push_back(lg);
            // Extend: UNH(E.rho, A.rho') in original local row numbers
            int32_t prev = t.j ? sel_[t.i][t.j - 1] : 0;
            ListDesc le;
            le.npick = t.rp; le.nkeep = t.alpha - t.rp; le.map = br.U[br.ucur];
            le.pick = bc.Prow[t.par]; le.append = br.E + prev;
            le.keep = bc.Qrow[t.par]; le.keep_out = br.U[1 - br.ucur];
            ops.lists.push_back(le);
        }
    }

    // ClearDown's second MAD: R' := R' + A.E * R   (RRF = [R'; R] in append order)
    void cd_mad2(Ops& ops) {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0 || t.r == 0) continue;
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            int32_t rest = bj - t.r - t.rp;
            if (rest == 0) continue;
            GemmDesc g;
            g.M = t.r; g.N = rest; g.K = t.rp; g.p = p_;
            g.A = bc.AE[t.par]; g.lda = bj;
            g.B = bc.DR[1 - bc.dcur] + (int64_t)t.r * bc.ld; g.ldb = bc.ld;
            g.C = bc.DR[1 - bc.dcur]; g.ldc = bc.ld;
            g.D = bc.DR[1 - bc.dcur]; g.ldd = bc.ld;
            push_gemm(ops, g, st_.cd_mad);
        }
    }

    // host bookkeeping once the layer's ClearDowns are complete
    void cd_commit() {
        for (auto& t : tasks_) {
            int32_t prev = t.j ? sel_[t.i][t.j - 1] : 0;
            sel_[t.i][t.j] = prev + t.rp;
            if (!t.active || t.rp == 0) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            rankc_[t.j] += t.rp;
            alpha_[t.i] -= t.rp;
            bc.dcur ^= 1;
            bc.gcur ^= 1;
            br.ucur ^= 1;
        }
    }

    // UpdateRow / UpdateRowTrafo step (3): X := A.M * V with V = rho' Z (and ADI for h = i)
    void ur3(Ops& pri, Bulk& bulk) {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            uint8_t* X = P_ + (bc.prow0 + t.r) * ldP_;
            int64_t c0 = C0_[t.j + 1];
            if (n_ - c0 > 0) {
                GemmDesc g;
                g.M = t.rp; g.N = (int32_t)(n_ - c0); g.K = t.rp; g.p = p_;
                g.A = bc.AM[t.par]; g.lda = bj;
                g.B = br.C[br.cur] + c0; g.ldb = br.ldC; g.brow = bc.Prow[t.par];
                g.D = X + c0; g.ldd = ldP_;
                push_split(pri, bulk, g, t.j, st_.ur_mad);
            }
            for (int h = 0; trafo_ && h <= t.i; ++h) {
                int32_t w = (h < t.i) ? sel_[h][t.j] : (t.j ? sel_[t.i][t.j - 1] : 0);
                if (w > 0) {
                    GemmDesc g;
                    g.M = t.rp; g.N = w; g.K = t.rp; g.p = p_;
                    g.A = bc.AM[t.par]; g.lda = bj;
                    g.B = br.K[br.cur] + R0_[h]; g.ldb = br.ldK; g.brow = bc.Prow[t.par];
                    g.D = X + n_ + R0_[h]; g.ldd = ldP_;
                    push_gemm(bulk.far, g, st_.urt_mad);
                }
                if (h == t.i) {
                    // V's identity columns (ADI) make X := A.M there
                    GatherDesc c;
                    c.rows = t.rp; c.cols = t.rp;
                    c.src = bc.AM[t.par]; c.lds = bj;
                    c.dst = X + n_ + R0_[h] + w; c.ldd = ldP_;
                    bulk.far.gather.push_back(c);
                    st_.gather_bytes += 2.0 * t.rp * t.rp;
                }
            }
        }
    }

    // step (4): S := B + A.E * X  (for h = i the stored M block is zero), RRF = append
    void ur4(Ops& pri, Bulk& bulk) {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0 || t.r == 0) continue;
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            uint8_t* Brow = P_ + bc.prow0 * ldP_;
            uint8_t* X = P_ + (bc.prow0 + t.r) * ldP_;
            int64_t c0 = C0_[t.j + 1];
            if (n_ - c0 > 0) {
                GemmDesc g;
                g.M = t.r; g.N = (int32_t)(n_ - c0); g.K = t.rp; g.p = p_;
                g.A = bc.AE[t.par]; g.lda = bj;
                g.B = X + c0; g.ldb = ldP_;
                g.C = Brow + c0; g.ldc = ldP_; g.D = Brow + c0; g.ldd = ldP_;
                push_split(pri, bulk, g, t.j, st_.ur_mad);
            }
            for (int h = 0; trafo_ && h <= t.i; ++h) {
                int32_t w = sel_[h][t.j];
                if (w == 0) continue;
                GemmDesc g;
                g.M = t.r; g.N = w; g.K = t.rp; g.p = p_;
                g.A = bc.AE[t.par]; g.lda = bj;
                g.B = X + n_ + R0_[h]; g.ldb = ldP_;
                g.C = Brow + n_ + R0_[h]; g.ldc = ldP_; g.D = Brow + n_ + R0_[h]; g.ldd = ldP_;
                push_gemm(bulk.far, g, st_.urt_mad);
            }
        }
    }

    // step (6): C := W + A.K * V with W = rho'-bar Z, written compacted to the other panel
    void ur6(Ops& pri, Bulk& bulk) {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0) continue;
            BR& br = rows_[t.i];
            BC& bc = cols_[t.j];
            int32_t bj = pr_.col_blocks[t.j];
            int32_t left = t.alpha - t.rp;
            if (left == 0) continue;
            int64_t c0 = C0_[t.j + 1];
            if (n_ - c0 > 0) {
                GemmDesc g;
                g.M = left; g.N = (int32_t)(n_ - c0); g.K = t.rp; g.p = p_;
                g.A = bc.AK[t.par]; g.lda = bj;
                g.B = br.C[br.cur] + c0; g.ldb = br.ldC; g.brow = bc.Prow[t.par];
                g.C = br.C[br.cur] + c0; g.ldc = br.ldC; g.crow = bc.Qrow[t.par];
                g.D = br.C[1 - br.cur] + c0; g.ldd = br.ldC;
                push_split(pri, bulk, g, t.j, st_.ur_mad);
            }
            for (int h = 0; trafo_ && h <= t.i; ++h) {
                int32_t w = (h < t.i) ? sel_[h][t.j] : (t.j ? sel_[t.i][t.j - 1] : 0);
                if (w > 0) {
                    GemmDesc g;
                    g.M = left; g.N = w; g.K = t.rp; g.p = p_;
                    g.A = bc.AK[t.par]; g.lda = bj;
                    g.B = br.K[br.cur] + R0_[h]; g.ldb = br.ldK; g.brow = bc.Prow[t.par];
                    g.C = br.K[br.cur] + R0_[h]; g.ldc = br.ldK; g.crow = bc.Qrow[t.par];
                    g.D = br.K[1 - br.cur] + R0_[h]; g.ldd = br.ldK;
                    push_gemm(bulk.far, g, st_.urt_mad);
                }
                if (h == t.i) {
                    // V is the identity on the new columns and W is zero there: K := A.K
                    GatherDesc c;
                    c.rows = left; c.cols = t.rp;
                    c.src = bc.AK[t.par]; c.lds = bj;
                    c.dst = br.K[1 - br.cur] + R0_[h] + w; c.ldd = br.ldK;
                    bulk.far.gather.push_back(c);
                    st_.gather_bytes += 2.0 * left * t.rp;
                }
            }
        }
    }

    void ur_commit() {
        for (auto& t : tasks_) {
            if (!t.active || t.rp == 0) continue;
            rows_[t.i].cur ^= 1;   // the compacted panels are now current
        }
    }

    // ------------------------------------------------------------ assembly, Step 2, Step 3
    int64_t rank() const {
        int64_t r = 0;
        for (int32_t x : rankc_) r += x;
        return r;
    }

    // allocate the result and emit the index sorts of the final orders
    bool assemble_lists(Result& res, Ops& ops) {
        r_ = rank();
        res.m = m_; res.n = n_; res.r = r_; res.p = p_;
        res.want = pr_.want;
        res.row_blocks = pr_.row_blocks;
        res.col_blocks = pr_.col_blocks;
        res.offR = (r_ + 15) / 16 * 16;
        res.offM = (res.offR + n_ - r_ + 15) / 16 * 16;
        // 64-byte aligned rows for the vector loads; [X R] only without the transformation
        res.ldP = ((trafo_ ? res.offM + r_ : res.offR + n_ - r_) + 63) / 64 * 64;
        res.ldK = r_;
        // the result in one allocation, the assembly maps in another (freed
        // with the plan): two allocations per problem, not ten
        Arena rb, mb;
        const size_t oPf = rb.take((size_t)std::max<int64_t>(keepR_ ? r_ * res.ldP : 0, 1));
        const size_t oKf = rb.take((size_t)std::max<int64_t>(trafo_ ? (m_ - r_) * r_ : 0, 1));
        const auto ilist = [](Arena& a, int64_t cnt) { return a.take(sizeof(int32_t) * std::max<int64_t>(cnt, 1)); };
        const size_t oU = ilist(rb, r_), oUb = ilist(rb, n_ - r_), oV = ilist(rb, r_), oVb = ilist(rb, m_ - r_);
        const size_t oRm = ilist(mb, r_), oCm = ilist(mb, n_ + r_), oKm = ilist(mb, r_), oOj = ilist(mb, r_);
        // GFECH_SEPARATE_BUFFERS=1: every piece its own allocation, so a
        // bounds-checking backend can tell an overrun of one into the next
        const char* sep_env = getenv("GFECH_SEPARATE_BUFFERS");
        const bool sep = sep_env && sep_env[0] == '1';
        std::map<size_t, uint8_t*> rp, mp;
        if (sep) {
            for (int a = 0; a < 2; ++a)
                for (auto& sl : (a ? mb : rb).slots) {
                    uint8_t* ptr = (uint8_t*)be_.alloc(std::max<size_t>(sl.second, 1));
                    if (!ptr) return false;
                    (a ? map_pieces_ : res.pieces).push_back(ptr);
                    (a ? mp : rp)[sl.first] = ptr;
                }
        } else {
            res.block = be_.alloc(rb.size);
            maps_ = be_.alloc(mb.size);
            if (!res.block || !maps_) return false;
        }
        const auto at = [&](size_t off) { return sep ? rp.at(off) : (uint8_t*)res.block + off; };
        const auto atm = [&](size_t off) { return sep ? mp.at(off) : (uint8_t*)maps_ + off; };
        res.Pfinal = at(oPf);
        res.Kfinal = at(oKf);
        res.upsilon = (int32_t*)at(oU);
        res.upsilon_bar = (int32_t*)at(oUb);
        res.varrho = (int32_t*)at(oV);
        res.varrho_bar = (int32_t*)at(oVb);
        rowmap_ = (int32_t*)atm(oRm);
        colmap_ = (int32_t*)atm(oCm);
        kmap_ = (int32_t*)atm(oKm);
        ordj_ = (int32_t*)atm(oOj);
        // block column offsets in the final orders
        rowoff_.assign(b_ + 1, 0);
        noff_.assign(b_ + 1, 0);
        for (int j = 0; j < b_; ++j) {
            rowoff_[j + 1] = rowoff_[j] + rankc_[j];
            noff_[j + 1] = noff_[j] + (pr_.col_blocks[j] - rankc_[j]);
        }
        soff_.assign(a_ + 1, 0);
        uoff_.assign(a_ + 1, 0);
        for (int h = 0; h < a_; ++h) {
            soff_[h + 1] = soff_[h] + (b_ ? sel_[h][b_ - 1] : 0);
            uoff_[h + 1] = uoff_[h] + alpha_[h];
        }
        for (int j = 0; j < b_; ++j) {
            BC& bc = cols_[j];
            int32_t rj = rankc_[j], nj = pr_.col_blocks[j] - rj;
            if (rj > 0) {
                SortDesc s;
                s.n = rj; s.vals = bc.Gam;
                s.mode = 1; s.add = 0; s.out = ordj_ + rowoff_[j];
                ops.sort.push_back(s);
                s.mode = 1; s.add = (int32_t)bc.prow0; s.out = rowmap_ + rowoff_[j];
                ops.sort.push_back(s);
                s.mode = 0; s.add = (int32_t)C0_[j]; s.out = colmap_ + rowoff_[j];
                ops.sort.push_back(s);
                s.out = res.upsilon + rowoff_[j];
                ops.sort.push_back(s);
            }
            if (nj > 0) {
                ListDesc l;
                l.npick = nj; l.add = (int32_t)C0_[j]; l.map = bc.Gbar[bc.gcur];
                l.append = colmap_ + r_ + noff_[j];
                ops.lists.push_back(l);
                l.append = res.upsilon_bar + noff_[j];
                ops.lists.push_back(l);
            }
        }
        for (int h = 0; h < a_; ++h) {
            BR& br = rows_[h];
            int32_t sh = soff_[h + 1] - soff_[h];
            if (sh > 0) {
                SortDesc s;
                s.n = sh; s.vals = br.E;
                if (trafo_) {
                    s.mode = 1; s.add = (int32_t)(n_ + R0_[h]); s.out = colmap_ + n_ + soff_[h];
                    ops.sort.push_back(s);
                    s.mode = 1; s.add = (int32_t)R0_[h]; s.out = kmap_ + soff_[h];
                    ops.sort.push_back(s);
                }
                s.mode = 0; s.add = (int32_t)R0_[h]; s.out = res.varrho + soff_[h];
                ops.sort.push_back(s);
            }
            if (alpha_[h] > 0) {
                ListDesc l;
                l.npick = alpha_[h]; l.add = (int32_t)R0_[h]; l.map = br.U[br.ucur];
                l.append = res.varrho_bar + uoff_[h];
                ops.lists.push_back(l);
            }
        }
        if (a_ == 0 || b_ == 0) {
            // degenerate shapes: every row non-selected / every column non-pivot
            std::vector<int32_t> io(std::max<int64_t>(m_, n_));
            std::iota(io.begin(), io.end(), 0);
            if (m_) be_.upload(res.varrho_bar, io.data(), sizeof(int32_t) * m_);
            if (n_) be_.upload(res.upsilon_bar, io.data(), sizeof(int32_t) * n_);
        }
        return true;
    }

    // PreClearUp + Copy for every block at once: gather the pivot matrix into
    // the final [X | R | M] layout (rows ordered by pivot column), then place
    // the diagonal remnants D_k.R.  RowLengthen (Step 2) is already done:
    // columns of rows selected later were never written and are zero.
    void repack(Result& res, Ops& ops) {
        if (r_ == 0 || !keepR_) return;
        // X, R and M to their column ranges (colmap_ lists the source columns of [X R M])
        const int64_t part[3][3] = {{0, 0, r_}, {r_, res.offR, n_ - r_}, {n_, res.offM, trafo_ ? r_ : 0}};
        for (const auto& q : part) {
            if (q[2] == 0) continue;
            GatherDesc g;
            g.rows = (int32_t)r_; g.cols = (int32_t)q[2];
            g.src = P_; g.lds = ldP_; g.srow = rowmap_; g.scol = colmap_ + q[0];
            g.dst = res.Pfinal + q[1]; g.ldd = res.ldP;
            ops.gather.push_back(g);
        }
        st_.gather_bytes += 2.0 * r_ * (n_ + (trafo_ ? r_ : 0));
        // the gaps before R and before M (and after R, up to the leading dimension, without M)
        const int64_t gap[2][2] = {{r_, res.offR}, {res.offR + n_ - r_, trafo_ ? res.offM : res.ldP}};
        for (const auto& q : gap) {
            if (q[1] == q[0]) continue;
            FillDesc f;
            f.rows = (int32_t)r_; f.cols = (int32_t)(q[1] - q[0]);
            f.dst = res.Pfinal + q[0]; f.ldd = res.ldP;
            ops.fill.push_back(f);
        }
    }

    void repack_diag(Result& res, Ops& ops) {
        if (!keepR_) return;
        for (int j = 0; j < b_; ++j) {
            BC& bc = cols_[j];
            int32_t rj = rankc_[j], nj = pr_.col_blocks[j] - rj;
            if (rj == 0 || nj == 0) continue;
            GatherDesc g;
            g.rows = rj; g.cols = nj;
            g.src = bc.DR[bc.dcur]; g.lds = bc.ld; g.srow = ordj_ + rowoff_[j];
            g.dst = res.Pfinal + rowoff_[j] * res.ldP + res.offR + noff_[j]; g.ldd = res.ldP;
            ops.gather.push_back(g);
        }
        // K: (m - r) x r, rows = the final non-selected rows of each block row,
        // columns = selected rows in ascending order (zero for block rows h > i)
        if (trafo_ && m_ - r_ > 0 && r_ > 0) {
            FillDesc f;
            f.rows = (int32_t)(m_ - r_); f.cols = (int32_t)r_;
            f.dst = res.Kfinal; f.ldd = res.ldK;
            ops.fill.push_back(f);
        }
    }

    void k_assemble(Result& res, Ops& ops) {
        if (!trafo_ || m_ - r_ == 0 || r_ == 0) return;
        for (int i = 0; i < a_; ++i) {
            BR& br = rows_[i];
            int32_t cols = soff_[i + 1];
            if (alpha_[i] == 0 || cols == 0) continue;
            GatherDesc g;
            g.rows = alpha_[i]; g.cols = cols;
            g.src = br.K[br.cur]; g.lds = br.ldK; g.scol = kmap_;
            g.dst = res.Kfinal + uoff_[i] * res.ldK; g.ldd = res.ldK;
            ops.gather.push_back(g);
            st_.gather_bytes += 2.0 * alpha_[i] * cols;
        }
    }

    // Step 3 (ClearUp), as a list of dependent launches.  Clearing the rows
    // of block columns j < k with the pivot rows of block column k is
    //     [R_{j, l>=k} | M_j] += X_jk * [R_{k, l>=k} | M_k]
    // for k from b down to 2 (Section 3, Step 3).  A pivot row of block column
    // k is zero in the pivot columns of every block column before k, so using
    // it never changes X_jk' for k' < k: the updates of a group G of
    // consecutive block columns can be applied together.  For each group
    // (taken from the right, about `group_rank` pivots each): first the
    // sequential clearing inside G, then one product for all rows above G
    // with inner dimension |pivots of G|:
    //     [R | M]_{rows above G} += X_{rows above G, G} * [R | M]_{rows of G}
    // which is the same sum the column-by-column order forms.
    void plan_clearup(Result& res, int64_t group_rank) {
        cu_steps_.clear();
        if (!keepR_) return;                            // the rank alone: no Step 3
        int k1 = b_;                                    // group = block columns [k0, k1)
        while (k1 > 1) {
            int k0 = k1 - 1;
            while (k0 > 0 && rowoff_[k1] - rowoff_[k0] < group_rank) --k0;
            if (rowoff_[k1] - rowoff_[k0] > group_rank && k0 < k1 - 1) ++k0;
            // inside the group, column by column
            for (int k = k1 - 1; k > k0; --k) {
                GemmDesc g;
                if (clearup_desc(res, k, rowoff_[k0], rowoff_[k], rowoff_[k], rowoff_[k + 1], k, g))
                    cu_steps_.push_back({g});
            }
            // every row above the group at once
            GemmDesc g;
            if (clearup_desc(res, k0, 0, rowoff_[k0], rowoff_[k0], rowoff_[k1], k0, g)) cu_steps_.push_back({g});
            k1 = k0;
        }
    }
    size_t clearup_steps() const { return cu_steps_.size(); }
    void clearup_step(size_t s, Ops& ops) {
        if (s >= cu_steps_.size()) return;
        for (const GemmDesc& g : cu_steps_[s]) push_gemm(ops, g, st_.cu_mad);
    }

    void release_maps() {
        be_.release(maps_);
        for (void* v : map_pieces_) be_.release(v);
        map_pieces_.clear();
        maps_ = nullptr;
        rowmap_ = colmap_ = kmap_ = ordj_ = nullptr;
    }

    size_t arena_bytes() const { return arena_bytes_; }

private:
    struct BR {
        size_t oC[2] = {0, 0}, oK[2] = {0, 0}, oU[2] = {0, 0}, oE = 0;
        uint8_t* C[2] = {nullptr, nullptr};
        uint8_t* K[2] = {nullptr, nullptr};
        int32_t* U[2] = {nullptr, nullptr};
        int32_t* E = nullptr;
        int64_t ldC = 0, ldK = 0;
        int cur = 0, ucur = 0;
    };
    struct BC {
        size_t oDR[2] = {0, 0}, oGbar[2] = {0, 0}, oGam = 0, oH = 0, oW = 0;
        size_t oAA[kScratchCopies] = {}, oAM[kScratchCopies] = {}, oAK[kScratchCopies] = {};
        size_t oProw[kScratchCopies] = {}, oQrow[kScratchCopies] = {}, oAE[kScratchCopies] = {};
        size_t oPcol = 0, oQcol = 0;
        uint8_t* DR[2] = {nullptr, nullptr};
        int32_t* Gbar[2] = {nullptr, nullptr};
        int32_t* Gam = nullptr;
        // by layer mod kScratchCopies (read by the bulk lane up to two layers late)
        uint8_t* AA[kScratchCopies] = {};
        uint8_t* AM[kScratchCopies] = {};
        uint8_t* AK[kScratchCopies] = {};
        int32_t* Prow[kScratchCopies] = {};
        int32_t* Qrow[kScratchCopies] = {};
        uint8_t* AE[kScratchCopies] = {};
        uint8_t *H = nullptr, *W = nullptr;
        int32_t *Pcol = nullptr, *Qcol = nullptr;
        int64_t cap = 0, ld = 0, ldW = 0, prow0 = 0;
        int dcur = 0, gcur = 0;
    };

    void push_gemm(Ops& ops, const GemmDesc& g, double& counter) {
        if (g.M <= 0 || g.N <= 0) return;
        ops.gemm.push_back(g);
        ops.gemm.back().kind = &counter == &st_.cd_mad    ? kGemmClearDown
                               : &counter == &st_.ur_mad  ? kGemmUpdateRow
                               : &counter == &st_.urt_mad ? kGemmUpdateRowTrafo
                               : &counter == &st_.cu_mad  ? kGemmClearUp
                                                          : kGemmOther;
        counter += (double)g.M * g.N * g.K;
    }

    // rows [rlo, rhi) of [X | R | M] += X[rows, plo:phi] * rows [plo, phi),
    // on the columns from block column kc's remnant to the end
    bool clearup_desc(Result& res, int kc, int64_t rlo, int64_t rhi, int64_t plo, int64_t phi, int, GemmDesc& g) {
        if (rhi - rlo <= 0 || phi - plo <= 0) return false;
        // from block column kc's remnant to the end of M, started at the 16-byte
        // boundary at or before it inside R: the pivot rows of block columns
        // >= kc are zero in every column of earlier block columns, so the
        // columns added on the left keep their values
        const int64_t c0u = res.offR + noff_[kc];
        const int64_t c0 = std::max<int64_t>(res.offR, c0u & ~(int64_t)15);
        const int64_t end = trafo_ ? res.offM + r_ : res.offR + n_ - r_;   // through M, or R alone
        const int64_t width = end - c0;
        if (c0u >= end) return false;
        g = GemmDesc();
        g.M = (int32_t)(rhi - rlo); g.N = (int32_t)width; g.K = (int32_t)(phi - plo); g.p = p_;
        g.A = res.Pfinal + rlo * res.ldP + plo; g.lda = res.ldP;
        g.B = res.Pfinal + plo * res.ldP + c0; g.ldb = res.ldP;
        g.C = res.Pfinal + rlo * res.ldP + c0; g.ldc = res.ldP;
        g.D = res.Pfinal + rlo * res.ldP + c0; g.ldd = res.ldP;
        return true;
    }

    // g covers the data columns [C0_{j+1}, n) of a product of task (i, j):
    // block column j + 1 goes to `pri`, the columns after it to `bulk`
    // columns [C0_[j + 1], C0_[j + 2]) to the priority lane, the next block
    // column to the bulk part's near set, the rest to its far set
    void push_split(Ops& pri, Bulk& bulk, const GemmDesc& g, int j, double& counter) {
        const int64_t e1 = std::min<int64_t>(g.N, C0_[j + 2] - C0_[j + 1]);
        const int64_t e2 = j + 3 <= b_ ? std::min<int64_t>(g.N, C0_[j + 3] - C0_[j + 1]) : g.N;
        const int64_t e3 = j + 4 <= b_ ? std::min<int64_t>(g.N, C0_[j + 4] - C0_[j + 1]) : g.N;
        const auto part = [&](Ops& ops, int64_t lo, int64_t hi) {
            if (hi <= lo) return;
            GemmDesc c = g;
            c.N = (int32_t)(hi - lo);
            c.B = g.B + lo;
            if (g.C) c.C = g.C + lo;
            c.D = g.D + lo;
            push_gemm(ops, c, counter);
        };
        part(pri, 0, e1);
        part(bulk.near, e1, e2);
        part(bulk.mid, e2, e3);
        part(bulk.far, e3, g.N);
    }

    Backend& be_;
    const Problem& pr_;
    Stats& st_;
    int a_ = 0, b_ = 0;
    int64_t m_ = 0, n_ = 0;
    int32_t p_ = 0;
    int32_t amax_ = 0;
    bool trafo_ = true;    // the transformation (K panels, M columns of P, UpdateRowTrafo, M in Step 3)
    bool keepR_ = true;    // the reduced remnant R (Step 3)
    std::vector<int64_t> R0_, C0_;
    std::vector<int32_t> alpha_, rankc_;
    std::vector<std::vector<int32_t>> sel_;   // sel_[h][j] = |E_{h,j}.rho|
    std::vector<BR> rows_;
    std::vector<BC> cols_;
    std::vector<TaskState> tasks_;
    std::vector<std::pair<size_t, size_t>> slots_, panel_slots_;
    size_t panel_bytes_ = 0;
    uint8_t* P_ = nullptr;
    int32_t* counts_ = nullptr;
    size_t oP_ = 0, arena_bytes_ = 0;
    int64_t prow_total_ = 0, ldP_ = 0, r_ = 0;
    void* maps_ = nullptr;   // the block the four maps below are carved from
    std::vector<void*> map_pieces_;   // or their separate allocations
    int32_t *rowmap_ = nullptr, *colmap_ = nullptr, *kmap_ = nullptr, *ordj_ = nullptr;
    std::vector<int64_t> rowoff_, noff_, soff_, uoff_;
    std::vector<std::vector<GemmDesc>> cu_steps_;
};

// GFECH_TRACE_MAD=<file>: every MAD launch of the engine is appended to the
// file, one line per descriptor: engine iteration, launch number, kind
// (GemmKind), M N K p, leading dimensions, flags and the operand addresses (a
// measurement aid: the shapes of a layer's launches can be replayed alone).
FILE* g_trace = nullptr;
int64_t g_trace_iter = 0, g_trace_launch = 0;
std::mutex g_trace_mu;     // engines of several threads (a server's size classes) may trace

void trace_gemm(const std::vector<GemmDesc>& ds) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (!g_trace) return;
    for (const GemmDesc& g : ds)
        fprintf(g_trace, "%lld %lld %d %d %d %d %d %lld %lld %lld %lld %d %p %p %p %p %p %p\n",
                (long long)g_trace_iter, (long long)g_trace_launch, g.kind, g.M, g.N, g.K, g.p, (long long)g.lda,
                (long long)g.ldb, (long long)g.ldc, (long long)g.ldd, g.flags, (const void*)g.A, (const void*)g.B,
                (const void*)g.C, (void*)g.D, (const void*)g.brow, (const void*)g.crow);
    ++g_trace_launch;
}

void flush(Backend& be, Ops& ops, Stats& st) {
    if (!ops.gather.empty()) { be.gather(ops.gather); st.launches++; }
    if (!ops.fill.empty()) { be.fill(ops.fill); st.launches++; }
    if (!ops.lists.empty()) { be.lists(ops.lists); st.launches++; }
    if (!ops.sort.empty()) { be.sort(ops.sort); st.launches++; }
    if (!ops.gemm.empty()) {
        // every buffer of the plan holds whole rows of its leading dimension
        for (GemmDesc& g : ops.gemm) g.flags |= kGemmRowsPadded;
        if (g_trace) trace_gemm(ops.gemm);
        be.gemm(ops.gemm);
        st.launches++;
        st.gemms += (int64_t)ops.gemm.size();
        for (const GemmDesc& g : ops.gemm)
            st.mad_bytes += (double)g.M * g.K + (double)g.K * g.N + (g.C ? 2.0 : 1.0) * g.M * g.N;
    }
    if (!ops.ech.empty()) { be.ech(ops.ech); st.launches++; }
    ops = Ops();
}

}  // namespace

// ============================================================================ engine

namespace {

enum Phase { kStep1, kAssemble, kClearUp, kFinished };

// capacity of the pivot-count pool: one int per block column of each active problem
constexpr size_t kCountsCap = 1 << 18;
// C panels at least this large are freed as soon as their problem leaves
// Step 1 (at the cost of one synchronisation), smaller ones with the rest
constexpr size_t kEarlyPanelFree = (size_t)1 << 30;

}  // namespace

struct Engine::Impl {
    struct Job {
        int64_t id = 0;
        Problem pr;
        Stats st;
        std::unique_ptr<Plan> plan;
        uint8_t* arena = nullptr;
        uint8_t* panels = nullptr;           // the C panels (freed when Step 1 ends)
        std::vector<void*> pieces, panel_pieces;
        size_t counts_off = 0, counts_n = 0;
        Phase phase = kStep1;
        bool cancel = false;
        int layer = 0;
        size_t cu_step = 0;
        std::unique_ptr<Result> res;
        size_t bytes = 0;
        int status = 0;
    };

    Impl(Backend& b, const Engine* e) : be(b), owner(e) {
        const char* tr = getenv("GFECH_TRACE_MAD");
        if (tr && tr[0]) {
            std::lock_guard<std::mutex> lk(g_trace_mu);
            if (!g_trace) {
                g_trace = fopen(tr, "a");
                g_trace_iter = g_trace_launch = 0;
                owns_trace = g_trace != nullptr;
            }
        }
        const char* ht = getenv("GFECH_HOST_TIMING");
        host_timing = ht && ht[0] == '1';
        const char* gr = getenv("GFECH_CLEARUP_GROUP");
        group_rank = gr ? std::max<int64_t>(1, atoll(gr)) : kClearUpGroup;
        counts = be.counts_buffer(kCountsCap);
        if (counts) holes.push_back({0, kCountsCap});
        hcounts.resize(kCountsCap);
    }
    ~Impl() {
        if (host_timing && ht_layers)
            fprintf(stderr, "gfech host timing: %lld layers, per layer %.1f us issue, %.1f us waiting for the "
                            "pivot counts, %.1f us after\n",
                    (long long)ht_layers, 1e6 * ht_pre / ht_layers, 1e6 * ht_wait / ht_layers,
                    1e6 * ht_post / ht_layers);
        if (host_timing && ht_layers)
            fprintf(stderr, "gfech host timing: issue by part (us per layer): wait and begin %.1f, extract %.1f, "
                            "ClearDown MADs %.1f, ECH %.1f, near set %.1f, UpdateRow (1) %.1f, rest %.1f\n",
                    1e6 * ht_seg[0] / ht_layers, 1e6 * ht_seg[1] / ht_layers, 1e6 * ht_seg[2] / ht_layers,
                    1e6 * ht_seg[3] / ht_layers, 1e6 * ht_seg[4] / ht_layers, 1e6 * ht_seg[5] / ht_layers,
                    1e6 * ht_seg[6] / ht_layers);
        if (host_timing)
            fprintf(stderr, "gfech host timing: after Step 1 (ms): assembly %.2f, ClearUp issue %.2f, finishing %.2f\n",
                    1e3 * ht_tail[0], 1e3 * ht_tail[1], 1e3 * ht_tail[2]);
        be.sync();
        for (auto& j : jobs) release(*j);
        if (counts) be.release_counts(counts);
        if (owns_trace) {
            std::lock_guard<std::mutex> lk(g_trace_mu);
            fclose(g_trace);
            g_trace = nullptr;
        }
    }
    bool owns_trace = false;
    // GFECH_HOST_TIMING=1: host time of Step 1 by phase, printed when the
    // engine ends (issue before the pivot-count read, the read's wait, the
    // rest of the layer)
    bool host_timing = false;
    double ht_pre = 0, ht_wait = 0, ht_post = 0;
    double ht_seg[7] = {0, 0, 0, 0, 0, 0, 0};   // the issue phase by part (see step())
    double ht_tail[3] = {0, 0, 0};              // assembly, ClearUp issue, finishing (with its wait)
    int64_t ht_layers = 0;

    Backend& be;
    const Engine* owner;
    Stats shared;
    std::vector<std::unique_ptr<Job>> jobs;
    Ops init_ops;              // the initial jobs of problems added since the last step
    std::vector<Done> done;
    int64_t next_id = 0;
    size_t bytes_in_use = 0;
    int mid_done = -1;         // lane 1's mark after the last bulk part issued (its mid set)
    int near_done = -1;        // lane 1's mark after that bulk part's near set
    int far_done = -1;         // lane 3's mark after its far set
    int far_wait = -1;         // the far set lane 0 waits for before the next layer's ClearDowns
    int u1_done = -1;          // lane 2's mark after this layer's UpdateRow (1) priority products
    Bulk b1, b3, b4, b6;       // the bulk part of the previous layer, not issued yet
    Ops u1;                    // this layer's UpdateRow (1) priority products
    int32_t* counts = nullptr;
    std::vector<std::pair<size_t, size_t>> holes;   // free ranges of the counts pool
    size_t counts_high = 0;
    std::vector<int32_t> hcounts;
    static constexpr int64_t kClearUpGroup = 16384;   // pivots per ClearUp group (GFECH_CLEARUP_GROUP)
    int64_t group_rank = kClearUpGroup;

    bool take_counts(size_t n, size_t* off) {
        n = std::max<size_t>(n, 1);
        for (auto& h : holes) {
            if (h.second >= n) {
                *off = h.first;
                h.first += n;
                h.second -= n;
                counts_high = std::max(counts_high, *off + n);
                return true;
            }
        }
        return false;
    }
    void give_counts(size_t off, size_t n) {
        n = std::max<size_t>(n, 1);
        holes.push_back({off, n});
        std::sort(holes.begin(), holes.end());
        std::vector<std::pair<size_t, size_t>> merged;
        for (auto& h : holes) {
            if (!merged.empty() && merged.back().first + merged.back().second == h.first) merged.back().second += h.second;
            else if (h.second) merged.push_back(h);
        }
        holes.swap(merged);
    }

    void release_panels(Job& j) {
        be.release(j.panels);
        for (void* v : j.panel_pieces) be.release(v);
        j.panels = nullptr;
        j.panel_pieces.clear();
    }

    void release(Job& j) {
        if (j.plan) j.plan->release_maps();
        be.release(j.arena);
        for (void* v : j.pieces) be.release(v);
        j.arena = nullptr;
        j.pieces.clear();
        release_panels(j);
        if (j.counts_n) give_counts(j.counts_off, j.counts_n);
        j.counts_n = 0;
        bytes_in_use -= j.bytes;
        j.bytes = 0;
    }

    // the near sets first, so the next layer's priority products wait only
    // for them (issue_near), then the mid sets (after the previous far sets,
    // which update their blocks too) and the far sets on lane 3 (issue_rest)
    void issue_near(int ready) {
        if (b1.empty() && b3.empty() && b4.empty() && b6.empty()) {
            // nothing new: a wait for the near set must cover every mid set issued so far
            near_done = mid_done;
            return;
        }
        be.set_lane(1);
        be.wait_mark(1, ready);
        flush(be, b1.near, shared);
        flush(be, b3.near, shared);
        flush(be, b4.near, shared);
        flush(be, b6.near, shared);
        near_done = be.mark(1);
        be.set_lane(0);
    }
    void issue_rest(int ready) {
        if (b1.empty() && b3.empty() && b4.empty() && b6.empty()) return;
        be.set_lane(1);
        if (far_done >= 0) be.wait_mark(1, far_done);
        flush(be, b1.mid, shared);
        flush(be, b3.mid, shared);
        flush(be, b4.mid, shared);
        flush(be, b6.mid, shared);
        mid_done = be.mark(1);
        be.set_lane(3);
        be.wait_mark(3, ready);
        flush(be, b1.far, shared);
        flush(be, b3.far, shared);
        flush(be, b4.far, shared);
        flush(be, b6.far, shared);
        far_done = be.mark(3);
        be.set_lane(0);
    }
    void issue_bulk(int ready) {
        issue_near(ready);
        issue_rest(ready);
    }
    // lane 0 waits for every bulk part issued so far
    void wait_bulk() {
        if (mid_done >= 0) be.wait_mark(0, mid_done);
        if (far_done >= 0) be.wait_mark(0, far_done);
    }

    void read_counts() {
        be.read_counts(hcounts.data(), counts, std::max<size_t>(counts_high, 1));
        shared.syncs++;
    }

    int64_t add(const Problem& pr, int* status) {
        std::unique_ptr<Job> j(new Job());
        j->pr = pr;
        j->plan.reset(new Plan(be, j->pr, j->st));
        const size_t sz = j->plan->plan_memory();
        j->counts_n = std::max<size_t>(j->plan->blockcols(), 1);
        if (!counts || !take_counts(j->counts_n, &j->counts_off)) {
            j->counts_n = 0;
            if (status) *status = 4;
            return -1;
        }
        // GFECH_SEPARATE_BUFFERS=1: every sub-buffer is its own allocation, so a
        // bounds-checking backend can tell any overrun of one buffer into the next
        const char* sep_env = getenv("GFECH_SEPARATE_BUFFERS");
        if (sep_env && sep_env[0] == '1') {
            std::map<size_t, uint8_t*> where, where_c;
            for (int arena = 0; arena < 2; ++arena) {
                for (auto& sl : arena ? j->plan->panel_slots() : j->plan->slots()) {
                    uint8_t* ptr = (uint8_t*)be.alloc(std::max<size_t>(sl.second, 1));
                    if (!ptr) {
                        release(*j);
                        if (status) *status = 4;
                        return -1;
                    }
                    (arena ? j->panel_pieces : j->pieces).push_back(ptr);
                    (arena ? where_c : where)[sl.first] = ptr;
                }
            }
            j->plan->bind([&](size_t off) { return where.at(off); }, [&](size_t off) { return where_c.at(off); },
                          counts + j->counts_off);
        } else {
            const size_t pb = j->plan->panel_bytes();
            j->arena = (uint8_t*)be.alloc(std::max<size_t>(sz - pb, 1));
            j->panels = (uint8_t*)be.alloc(std::max<size_t>(pb, 1));
            if (!j->arena || !j->panels) {
                release(*j);
                if (status) *status = 4;
                return -1;
            }
            uint8_t* base = j->arena;
            uint8_t* cbase = j->panels;
            j->plan->bind([base](size_t off) { return base + off; }, [cbase](size_t off) { return cbase + off; },
                          counts + j->counts_off);
        }
        j->bytes = owner->footprint(j->pr);
        bytes_in_use += j->bytes;
        j->plan->init(init_ops);
        j->id = next_id++;
        j->phase = j->plan->layers() > 0 ? kStep1 : kAssemble;
        jobs.push_back(std::move(j));
        if (status) *status = 0;
        return jobs.back()->id;
    }

    void fail_all(int rc) {
        be.sync();
        for (auto& j : jobs) {
            release(*j);
            Done d;
            d.id = j->id;
            d.status = rc;
            done.push_back(std::move(d));
        }
        jobs.clear();
    }

    // cancelled problems: the bulk part issued last may name their buffers,
    // so every lane drains before their memory is freed
    void drop_cancelled() {
        bool any = false;
        for (auto& j : jobs) any = any || j->cancel;
        if (!any) return;
        issue_bulk(be.mark(0));
        wait_bulk();
        be.sync();
        b1 = Bulk(); b3 = Bulk(); b4 = Bulk(); b6 = Bulk();
        std::vector<std::unique_ptr<Job>> keep;
        for (auto& j : jobs) {
            if (!j->cancel) {
                keep.push_back(std::move(j));
                continue;
            }
            release(*j);
            Done d;
            d.id = j->id;
            d.status = kCancelled;
            done.push_back(std::move(d));
        }
        jobs.swap(keep);
    }

    size_t step() {
        if (owns_trace) {
            std::lock_guard<std::mutex> lk(g_trace_mu);
            ++g_trace_iter;
        }
        if (be.error()) {
            fail_all(be.error());
            return 0;
        }
        drop_cancelled();
        if (jobs.empty()) {
            flush(be, init_ops, shared);
            return 0;
        }
        Ops ops;
        flush(be, init_ops, shared);
        std::vector<Plan*> s1;
        for (auto& j : jobs)
            if (j->phase == kStep1) s1.push_back(j->plan.get());
        // ---- Step 1: one layer of every problem in it (see the header comment for the lanes)
        if (!s1.empty()) {
            const auto h0 = std::chrono::steady_clock::now();
            auto h1 = h0, h2 = h0, hp = h0;
            int seg = 0;
            const auto tick = [&] {
                if (!host_timing) return;
                const auto t = std::chrono::steady_clock::now();
                ht_seg[seg++] += std::chrono::duration<double>(t - hp).count();
                hp = t;
            };
            // the bulk part issued two layers back reads the scratch copy this
            // layer's ClearDowns write: its mid set is behind the near set lane 0
            // waited for in the previous layer, its far set is waited for here
            if (far_wait >= 0) be.wait_mark(0, far_wait);
            far_wait = far_done;
            for (size_t q = 0; q < jobs.size(); ++q)
                if (jobs[q]->phase == kStep1) jobs[q]->plan->begin_layer(jobs[q]->layer);
            tick();
            for (Plan* pl : s1) pl->cd_extract(ops);
            flush(be, ops, shared);
            tick();
            for (Plan* pl : s1) pl->cd_mad(ops);
            flush(be, ops, shared);
            tick();
            // the previous layer's bulk part starts after this layer's ClearDown
            // MADs and is issued after this layer's ECHs, so the ECHs (one
            // workgroup each) reach the device first: issued behind a large
            // product, an ECH would wait for that product's last tiles
            const int ready = be.mark(0);
            bool any = false;
            for (Plan* pl : s1) { pl->cd_ech(ops, false); any = any || pl->any_ech(); }
            flush(be, ops, shared);
            tick();
            issue_near(ready);
            tick();
            // UpdateRow (1)'s priority products overwrite the near set's columns
            // and need nothing this layer's ECH computes: lane 2 runs them beside
            // the ECH, issued before the mid and far sets so that they reach the
            // device ahead of them (their bulk part joins the next layer's)
            Bulk b1n;
            for (Plan* pl : s1) pl->ur1(u1, b1n);
            u1_done = -1;
            if (!u1.empty()) {
                be.set_lane(2);
                be.wait_mark(2, ready);
                if (near_done >= 0) be.wait_mark(2, near_done);
                flush(be, u1, shared);
                u1_done = be.mark(2);
                be.set_lane(0);
            }
            tick();
            issue_rest(ready);
            tick();
            b1 = std::move(b1n);
            for (Plan* pl : s1) pl->clear_counts();
            h1 = std::chrono::steady_clock::now();
            if (any) {
                read_counts();
                if (be.error()) { fail_all(be.error()); return 0; }
                bool again = false;
                for (auto& j : jobs)
                    if (j->phase == kStep1) again = j->plan->absorb_counts(hcounts.data() + j->counts_off, false) || again;
                if (again) {
                    // the rows left unselected: reduced by the pivots found, are
                    // they zero after the leading columns?  Only where not, the
                    // ECH runs again on all of H
                    for (Plan* pl : s1) pl->cd_tail(ops);
                    flush(be, ops, shared);
                    std::vector<Backend::RangeDesc> rd;
                    for (Plan* pl : s1) pl->tail_ranges(rd);
                    std::vector<int64_t> nz;
                    be.count_out_of_range_many(rd, nz);
                    shared.syncs++;
                    if (be.error()) { fail_all(be.error()); return 0; }
                    size_t pos = 0;
                    again = false;
                    for (Plan* pl : s1) again = pl->absorb_tail(nz, pos) || again;
                }
                if (again) {
                    for (Plan* pl : s1) pl->cd_ech(ops, true);
                    flush(be, ops, shared);
                    read_counts();
                    if (be.error()) { fail_all(be.error()); return 0; }
                    for (auto& j : jobs)
                        if (j->phase == kStep1) j->plan->absorb_counts(hcounts.data() + j->counts_off, true);
                }
            }
            h2 = std::chrono::steady_clock::now();
            // The priority products below read what UpdateRow (1) wrote on lane 2
            // (after the previous bulk part's near set, whose columns they
            // overwrite).  That bulk part's far set (blocks after those) may
            // still run: nothing on this lane touches its columns before the
            // next layer's near set, which lane 1 runs after it, and the
            // scratch it reads is the copy of two layers back.
            if (u1_done >= 0) be.wait_mark(0, u1_done);
            else if (near_done >= 0) be.wait_mark(0, near_done);
            // Fewer launches on the chain: UpdateRow step (3) needs nothing
            // ClearDown's remaining parts produce and shares their launch; the
            // second MAD of ClearDown (which reads the remnant product) and steps
            // (4) (which reads step (3)) and (6) touch disjoint data and share
            // the next one.  The second MAD is planned before cd_commit, which
            // swaps the remnant buffers it names.
            for (Plan* pl : s1) pl->cd_post(ops);
            for (Plan* pl : s1) pl->ur3(ops, b3);
            flush(be, ops, shared);
            for (Plan* pl : s1) pl->cd_mad2(ops);
            for (Plan* pl : s1) pl->cd_commit();
            for (Plan* pl : s1) pl->ur4(ops, b4);
            for (Plan* pl : s1) pl->ur6(ops, b6);
            flush(be, ops, shared);
            for (Plan* pl : s1) pl->ur_commit();
            if (host_timing) {
                const auto h3 = std::chrono::steady_clock::now();
                ht_pre += std::chrono::duration<double>(h1 - h0).count();
                ht_wait += std::chrono::duration<double>(h2 - h1).count();
                ht_post += std::chrono::duration<double>(h3 - h2).count();
                ht_layers++;
            }
            shared.layers++;
            bool finished = false;
            for (auto& j : jobs) {
                if (j->phase != kStep1) continue;
                j->st.layers++;
                if (++j->layer >= j->plan->layers()) {
                    j->phase = kAssemble;
                    finished = true;
                }
            }
            // a problem leaving Step 1 needs its last bulk part before the assembly
            if (finished) {
                issue_bulk(be.mark(0));
                wait_bulk();
                // its C panels are not read again: large ones are freed now, so
                // that the result can take their place (the lanes drain first)
                bool big = false;
                for (auto& j : jobs)
                    if (j->phase == kAssemble && j->plan->panel_bytes() >= kEarlyPanelFree) big = true;
                if (big) {
                    be.sync();
                    for (auto& j : jobs)
                        if (j->phase == kAssemble) release_panels(*j);
                }
            }
        } else {
            issue_bulk(be.mark(0));
            wait_bulk();
        }
        if (be.error()) { fail_all(be.error()); return 0; }

        // ---- assembly of the result (and Step 2, implicit), then Step 3's plan
        const auto ha = std::chrono::steady_clock::now();
        std::vector<Job*> asmj;
        for (auto& j : jobs)
            if (j->phase == kAssemble) asmj.push_back(j.get());
        if (!asmj.empty()) {
            for (Job* j : asmj) {
                j->res.reset(new Result());
                j->res->be = &be;
                if (!j->plan->assemble_lists(*j->res, ops)) j->status = 4;
            }
            flush(be, ops, shared);
            for (Job* j : asmj) if (!j->status) j->plan->repack(*j->res, ops);
            flush(be, ops, shared);
            for (Job* j : asmj) if (!j->status) j->plan->repack_diag(*j->res, ops);
            flush(be, ops, shared);
            for (Job* j : asmj) if (!j->status) j->plan->k_assemble(*j->res, ops);
            flush(be, ops, shared);
            for (Job* j : asmj) {
                if (!j->status) j->plan->plan_clearup(*j->res, group_rank);
                j->phase = j->status ? kFinished : kClearUp;
                j->cu_step = 0;
            }
        }
        // ---- Step 3: the next ClearUp launch of every problem in it
        const auto hc = std::chrono::steady_clock::now();
        bool cu = false;
        for (auto& j : jobs) {
            if (j->phase != kClearUp) continue;
            if (j->cu_step < j->plan->clearup_steps()) {
                j->plan->clearup_step(j->cu_step++, ops);
                cu = true;
            }
        }
        if (cu) flush(be, ops, shared);
        for (auto& j : jobs)
            if (j->phase == kClearUp && j->cu_step >= j->plan->clearup_steps()) j->phase = kFinished;

        // ---- finished problems: their work must be complete before their memory is reused
        const auto hf = std::chrono::steady_clock::now();
        bool fin = false;
        for (auto& j : jobs) fin = fin || j->phase == kFinished;
        if (fin) {
            be.sync();
            const int rc = be.error();
            std::vector<std::unique_ptr<Job>> keep;
            for (auto& j : jobs) {
                if (j->phase != kFinished) {
                    keep.push_back(std::move(j));
                    continue;
                }
                release(*j);
                Done d;
                d.id = j->id;
                d.status = rc ? rc : j->status;
                if (!d.status) {
                    Stats st = j->st;
                    st.launches = shared.launches;
                    st.gemms = shared.gemms;
                    st.mad_bytes = shared.mad_bytes;
                    st.syncs = shared.syncs;
                    j->res->stats = st;
                    d.result = std::move(j->res);
                }
                done.push_back(std::move(d));
            }
            jobs.swap(keep);
        }
        if (host_timing) {
            const auto he = std::chrono::steady_clock::now();
            ht_tail[0] += std::chrono::duration<double>(hc - ha).count();
            ht_tail[1] += std::chrono::duration<double>(hf - hc).count();
            ht_tail[2] += std::chrono::duration<double>(he - hf).count();
        }
        return jobs.size();
    }
};

Engine::Engine(Backend& be) : impl_(new Impl(be, this)) {}
Engine::~Engine() = default;

size_t Engine::footprint(const Problem& pr) const {
    Stats st;
    Plan plan(impl_->be, pr, st);
    size_t bytes = plan.plan_memory() + kAlign;
    // the result (at most rank min(m, n)) and the assembly maps
    const size_t r = (size_t)std::min(pr.m, pr.n);
    if (pr.want == kWantAll)
        bytes += r * (size_t)((pr.n + (int64_t)r + 32 + 63) / 64 * 64) + (size_t)(pr.m - (int64_t)r) * r;
    else if (pr.want == kWantRref)
        bytes += r * (size_t)((pr.n + 16 + 63) / 64 * 64);
    bytes += sizeof(int32_t) * (size_t)(3 * pr.m + 3 * pr.n + 4 * r) + 16 * kAlign;
    return bytes;
}
int64_t Engine::add(const Problem& pr, int* status) { return impl_->add(pr, status); }
size_t Engine::step() { return impl_->step(); }
void Engine::cancel(int64_t id) {
    for (auto& j : impl_->jobs)
        if (j->id == id) j->cancel = true;
}
size_t Engine::active() const { return impl_->jobs.size(); }
size_t Engine::bytes_in_use() const { return impl_->bytes_in_use; }
std::vector<Engine::Done> Engine::take_done() {
    std::vector<Done> d;
    d.swap(impl_->done);
    return d;
}
const Stats& Engine::totals() const { return impl_->shared; }

int run_chief(Backend& be, const std::vector<Problem>& probs, std::vector<std::unique_ptr<Result>>& out,
              std::string* err, int profile, int64_t timeout_ms) {
    const auto t0 = std::chrono::steady_clock::now();
    if (profile) {
        be.take_profile();
        be.set_profile(profile);
    }
    std::vector<std::unique_ptr<Result>> res(probs.size());
    int rc = 0;
    {
        Engine eng(be);
        std::vector<int64_t> ids;
        for (const Problem& pr : probs) {
            int st = 0;
            const int64_t id = eng.add(pr, &st);
            if (id < 0) {
                if (err) *err = "device allocation of the block arena failed";
                rc = st ? st : 4;
                break;
            }
            ids.push_back(id);
        }
        bool cancelled = false;
        // GFECH_HOST_TIMING=1: host time of the call by part (planning, each
        // engine iteration, the end), printed when the call ends
        const char* ht = getenv("GFECH_HOST_TIMING");
        const bool timing = ht && ht[0] == '1';
        auto tp = std::chrono::steady_clock::now();
        std::vector<double> parts;
        if (timing) parts.push_back(std::chrono::duration<double>(tp - t0).count());
        while (!rc && eng.active()) {
            if (timeout_ms > 0 && !cancelled &&
                std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms)) {
                for (int64_t id : ids) eng.cancel(id);
                cancelled = true;
            }
            eng.step();
            if (timing) {
                const auto t = std::chrono::steady_clock::now();
                parts.push_back(std::chrono::duration<double>(t - tp).count());
                tp = t;
            }
        }
        if (timing) {
            fprintf(stderr, "gfech call timing (ms): %zu problems, planning %.2f, iterations", probs.size(),
                    1e3 * parts[0]);
            for (size_t k = 1; k < parts.size() && k <= 12; ++k) fprintf(stderr, " %.2f", 1e3 * parts[k]);
            if (parts.size() > 13) fprintf(stderr, " ... (%zu)", parts.size() - 1);
            fprintf(stderr, "\n");
        }
        for (auto& d : eng.take_done()) {
            if (d.status && !rc) {
                rc = d.status;
                if (err)
                    *err = rc == 4 ? "device allocation of the result failed"
                           : rc == kCancelled ? "cancelled by the watchdog"
                                              : "device error";
            }
            if (d.result && d.id < (int64_t)res.size()) res[(size_t)d.id] = std::move(d.result);
        }
        if (!rc) {
            be.sync();
            rc = be.error();
            if (rc && err) *err = "device error";
        }
    }
    Backend::Profile prof;
    if (profile) {
        prof = be.take_profile();
        be.set_profile(0);
    }
    if (rc) return rc;
    for (size_t q = 0; q < res.size(); ++q) {
        if (!res[q]) return 6;
        for (int k = 0; k < 3; ++k) {
            res[q]->stats.kernel_ms[k] = prof.ms[k];
            res[q]->stats.kernel_launches[k] = prof.launches[k];
            res[q]->stats.kernel_mac[k] = prof.mac[k];
        }
        out.push_back(std::move(res[q]));
    }
    return 0;
}

}  // namespace gfech
