// C ABI of libgfech (declared in include/gfech.h): argument checks, host /
// device staging, block-size choice and the result getters.  All arithmetic
// runs in the backend's kernels through the Chief.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gfech.h"
#include "backend.h"
#include "chief.h"

namespace gfech {
// Provided by the backend translation unit linked into the library: the
// shared instance of the plain calls, and further instances (own streams,
// memory cache and lock) for the server's size classes.  Instances are
// never destroyed: results keep pointers to the instance that made them.
Backend* backend_instance(std::string* err);
Backend* backend_acquire(std::string* err);
void backend_release(Backend* be);
}  // namespace gfech

struct gfech_result {
    std::unique_ptr<gfech::Result> r;
};

namespace {

thread_local std::string g_last_error;

gfech_status fail(gfech_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

bool is_prime(uint32_t p) {
    if (p < 2) return false;
    for (uint32_t d = 2; d * d <= p; ++d)
        if (p % d == 0) return false;
    return true;
}

// Blocking (Section 3.1).  An installed table of tuned block sizes
// (gfech_set_blocking) takes precedence; without one, up to 512 x 512 the
// whole matrix is one block (one ECH job), and larger matrices get blocks of
// 256 rows and 2048 columns: the ECH jobs on the critical path stay short
// (their cost grows with the rows of a block, and a ClearDown whose rows all
// become pivots in the leading columns finishes the remaining columns with
// one product), while UpdateRow's products get an inner dimension of up to
// 2048 pivots per block column, where the MFMA kernel runs several times
// faster than at 512.
std::mutex g_table_mu;
std::vector<gfech_blocking> g_table;

void choose_blocks(int64_t m, int64_t n, const gfech_opts* o, std::vector<int32_t>& a, std::vector<int32_t>& b) {
    const int64_t single = 512;
    int64_t br = (o && o->block_rows > 0) ? o->block_rows : 0;
    int64_t bc = (o && o->block_cols > 0) ? o->block_cols : 0;
    if (!br && !bc) {
        std::lock_guard<std::mutex> lk(g_table_mu);
        for (const gfech_blocking& t : g_table)
            if (std::max(m, n) <= t.max_dim) {
                br = t.block_rows;
                bc = t.block_cols;
                break;
            }
    }
    if (!br && !bc) {
        if (m <= single && n <= single) {
            br = m;
            bc = n;
        } else {
            br = 256;
            bc = 2048;
        }
    } else if (!br) {
        br = bc;
    } else if (!bc) {
        bc = br;
    }
    a = gfech::even_blocks(m, br);
    b = gfech::even_blocks(n, bc);
}

gfech_status check_common(int64_t m, int64_t n, int64_t lda, uint32_t p, const void* A) {
    if (m < 0 || n < 0) return fail(GFECH_E_ARG, "negative size");
    if (m > INT32_MAX || n > INT32_MAX || m + n > INT32_MAX) return fail(GFECH_E_TOO_BIG, "dimension too large");
    if (m > 0 && n > 0 && (!A || lda < n)) return fail(GFECH_E_ARG, "null input or lda < n");
    if (p > 251 || !is_prime(p)) return fail(GFECH_E_FIELD, "p must be a prime <= 251");
    return GFECH_OK;
}

gfech_status check_variant(const gfech_opts* o) {
    if (o && (o->variant < GFECH_WANT_RREF_T || o->variant > GFECH_WANT_RANK))
        return fail(GFECH_E_ARG, "unknown variant");
    return GFECH_OK;
}

int32_t variant_of(const gfech_opts* o) { return o ? o->variant : GFECH_WANT_RREF_T; }

// the result includes R (and E) / M, K (and T)
bool has_R(const gfech::Result& R) { return R.want != gfech::kWantRank; }
bool has_T(const gfech::Result& R) { return R.want == gfech::kWantAll; }

// the status of a planner / backend error code
gfech_status status_of(int rc) {
    return rc == 0 ? GFECH_OK : rc == 4 ? GFECH_E_NOMEM : rc == gfech::kCancelled ? GFECH_E_CANCELLED : GFECH_E_DEVICE;
}

gfech::Backend* get_backend(gfech_status* st) {
    std::string err;
    gfech::Backend* be = gfech::backend_instance(&err);
    if (!be) *st = fail(GFECH_E_DEVICE, err.empty() ? "no device backend" : err);
    return be;
}

// run a set of problems whose inputs are already in backend memory
gfech_status run(gfech::Backend* be, std::vector<gfech::Problem>& probs, gfech_result** outs,
                 const gfech_opts* opts) {
    std::vector<std::unique_ptr<gfech::Result>> res;
    std::string err;
    int rc = gfech::run_chief(*be, probs, res, &err, opts ? opts->profile : 0, opts ? opts->timeout_ms : 0);
    if (rc) return fail(status_of(rc), err);
    for (size_t q = 0; q < res.size(); ++q) {
        outs[q] = new gfech_result();
        outs[q]->r = std::move(res[q]);
    }
    return GFECH_OK;
}

gfech_status echelonise_impl(const uint8_t* A, bool on_device, int64_t m, int64_t n, int64_t lda, uint32_t p,
                             const gfech_opts* opts, void* stream, gfech_result** out) {
    if (!out) return fail(GFECH_E_ARG, "out is NULL");
    *out = nullptr;
    gfech_status st = check_common(m, n, lda, p, A);
    if (st) return st;
    if ((st = check_variant(opts))) return st;
    bool check = !(opts && opts->skip_range_check);
    if (!on_device && check) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (A[i * lda + j] >= p) return fail(GFECH_E_RANGE, "entry >= p");
    }
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    const uint8_t* dA = A;
    void* staged = nullptr;
    int64_t ld = lda;
    if (!on_device && m > 0 && n > 0) {
        staged = be->alloc((size_t)(m * n));
        if (!staged) return fail(GFECH_E_NOMEM, "device allocation of the input failed");
        if (lda == n) {
            be->upload(staged, A, (size_t)(m * n));
        } else {
            std::vector<uint8_t> tmp((size_t)(m * n));
            for (int64_t i = 0; i < m; ++i) memcpy(tmp.data() + i * n, A + i * lda, (size_t)n);
            be->upload(staged, tmp.data(), (size_t)(m * n));
        }
        dA = (const uint8_t*)staged;
        ld = n;
    } else if (on_device && check && m > 0 && n > 0) {
        int64_t bad = be->count_out_of_range(A, m, n, lda, (int32_t)p);
        if (bad != 0) {
            be->set_stream(nullptr);
            return fail(bad > 0 ? GFECH_E_RANGE : GFECH_E_DEVICE, bad > 0 ? "entry >= p" : "device error");
        }
    }
    std::vector<gfech::Problem> probs(1);
    probs[0].A = dA;
    probs[0].m = m;
    probs[0].n = n;
    probs[0].lda = ld;
    probs[0].p = (int32_t)p;
    probs[0].want = variant_of(opts);
    choose_blocks(m, n, opts, probs[0].row_blocks, probs[0].col_blocks);
    st = run(be, probs, out, opts);
    if (staged) be->release(staged);
    be->set_stream(nullptr);
    return st;
}

// GF(2) input packed in 64-bit words: unpacked on the device straight into
// the planner's block-row panels (one byte per entry), then the byte path
// over p = 2
gfech_status echelonise_gf2_impl(const uint64_t* A, bool on_device, int64_t m, int64_t n, int64_t ldw,
                                 const gfech_opts* opts, void* stream, gfech_result** out) {
    if (!out) return fail(GFECH_E_ARG, "out is NULL");
    *out = nullptr;
    if (m < 0 || n < 0 || ldw < 0) return fail(GFECH_E_ARG, "negative size");
    const int64_t words = (n + 63) / 64;
    if (m > 0 && n > 0 && (!A || ldw < words)) return fail(GFECH_E_ARG, "null input or ldw < ceil(n / 64)");
    gfech_status st = check_common(m, n, n, 2, A);
    if (st) return st;
    if ((st = check_variant(opts))) return st;
    const bool check = !(opts && opts->skip_range_check);
    if (!on_device && check && n % 64 && m > 0) {
        const uint64_t mask = ~((1ull << (n % 64)) - 1);
        for (int64_t i = 0; i < m; ++i)
            if (A[i * ldw + n / 64] & mask) return fail(GFECH_E_RANGE, "a pad bit past column n - 1 is set");
    }
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    const uint64_t* packed = A;
    int64_t ld = ldw;
    void* staged = nullptr;
    if (m > 0 && n > 0) {
        if (!on_device) {
            staged = be->alloc((size_t)(m * words) * 8);
            if (!staged) return fail(GFECH_E_NOMEM, "device allocation of the input failed");
            if (ldw == words) {
                be->upload(staged, A, (size_t)(m * words) * 8);
            } else {
                std::vector<uint64_t> tmp((size_t)(m * words));
                for (int64_t i = 0; i < m; ++i) memcpy(tmp.data() + i * words, A + i * ldw, (size_t)words * 8);
                be->upload(staged, tmp.data(), tmp.size() * 8);
            }
            packed = (const uint64_t*)staged;
            ld = words;
        } else if (check) {
            const int64_t bad = be->count_gf2_pad(A, m, n, ldw);
            if (bad != 0) {
                be->set_stream(nullptr);
                return fail(bad > 0 ? GFECH_E_RANGE : GFECH_E_DEVICE,
                            bad > 0 ? "a pad bit past column n - 1 is set" : "device error");
            }
        }
    }
    std::vector<gfech::Problem> probs(1);
    probs[0].packed = packed;
    probs[0].ldw = ld;
    probs[0].m = m;
    probs[0].n = n;
    probs[0].lda = std::max<int64_t>(n, 1);
    probs[0].p = 2;
    probs[0].want = variant_of(opts);
    choose_blocks(m, n, opts, probs[0].row_blocks, probs[0].col_blocks);
    st = run(be, probs, out, opts);
    be->release(staged);
    be->set_stream(nullptr);
    return st;
}

template <typename T>
gfech_status download_list(gfech::Backend* be, const int32_t* src, int64_t count, T* dst) {
    if (count == 0) return GFECH_OK;
    std::vector<int32_t> tmp((size_t)count);
    be->download(tmp.data(), src, sizeof(int32_t) * (size_t)count);
    for (int64_t i = 0; i < count; ++i) dst[i] = (T)tmp[(size_t)i];
    return GFECH_OK;
}

gfech_status download_matrix(gfech::Backend* be, const uint8_t* src, int64_t lds, int64_t rows, int64_t cols,
                             uint8_t* dst, int64_t ldd) {
    if (rows == 0 || cols == 0) return GFECH_OK;
    if (lds == cols && ldd == cols) {
        be->download(dst, src, (size_t)(rows * cols));
        return GFECH_OK;
    }
    std::vector<uint8_t> tmp((size_t)(rows * lds));
    be->download(tmp.data(), src, (size_t)((rows - 1) * lds + cols));
    for (int64_t i = 0; i < rows; ++i) memcpy(dst + i * ldd, tmp.data() + i * lds, (size_t)cols);
    return GFECH_OK;
}

void expand_rref_ops(const gfech::Result& R, uint8_t* E, int64_t lde, gfech::Backend* be) {
    int64_t r = R.r, n = R.n;
    if (r == 0 || n == 0) return;
    std::vector<gfech::FillDesc> f(2);
    f[0].rows = (int32_t)r; f[0].cols = (int32_t)n; f[0].dst = E; f[0].ldd = lde; f[0].value = 0;
    be->fill({f[0]});
    f[1].rows = (int32_t)r; f[1].dst = E; f[1].ldd = lde; f[1].diag_value = 1; f[1].dcol = R.upsilon;
    be->fill({f[1]});
    if (n - r > 0) {
        gfech::GatherDesc g;
        g.rows = (int32_t)r; g.cols = (int32_t)(n - r); g.neg_p = R.p;
        g.src = R.Pfinal + R.offR; g.lds = R.ldP;
        g.dst = E; g.ldd = lde; g.dcol = R.upsilon_bar;
        be->gather({g});
    }
}

void expand_transform_ops(const gfech::Result& R, uint8_t* T, int64_t ldt, gfech::Backend* be) {
    int64_t r = R.r, m = R.m;
    if (m == 0) return;
    gfech::FillDesc z;
    z.rows = (int32_t)m; z.cols = (int32_t)m; z.dst = T; z.ldd = ldt; z.value = 0;
    be->fill({z});
    if (r > 0) {
        gfech::GatherDesc g;
        g.rows = (int32_t)r; g.cols = (int32_t)r; g.neg_p = R.p;
        g.src = R.Pfinal + R.offM; g.lds = R.ldP;
        g.dst = T; g.ldd = ldt; g.dcol = R.varrho;
        be->gather({g});
        if (m - r > 0) {
            gfech::GatherDesc k;
            k.rows = (int32_t)(m - r); k.cols = (int32_t)r;
            k.src = R.Kfinal; k.lds = R.ldK;
            k.dst = T + r * ldt; k.ldd = ldt; k.dcol = R.varrho;
            be->gather({k});
        }
    }
    if (m - r > 0) {
        gfech::FillDesc id;
        id.rows = (int32_t)(m - r); id.dst = T + r * ldt; id.ldd = ldt; id.diag_value = 1; id.dcol = R.varrho_bar;
        be->fill({id});
    }
}

}  // namespace

extern "C" {

gfech_status gfech_echelonise_u8(const uint8_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p,
                                 const gfech_opts* opts, gfech_result** out) {
    return echelonise_impl(A, false, m, n, lda, p, opts, nullptr, out);
}

gfech_status gfech_echelonise_u8_dev(const uint8_t* A_dev, int64_t m, int64_t n, int64_t lda, uint32_t p,
                                     const gfech_opts* opts, void* stream, gfech_result** out) {
    return echelonise_impl(A_dev, true, m, n, lda, p, opts, stream, out);
}

gfech_status gfech_set_blocking(const gfech_blocking* table, int64_t count) {
    if (count < 0 || (count > 0 && !table)) return fail(GFECH_E_ARG, "bad blocking table");
    for (int64_t t = 0; t < count; ++t) {
        if (table[t].max_dim <= 0 || table[t].block_rows < 0 || table[t].block_cols < 0)
            return fail(GFECH_E_ARG, "bad blocking table entry");
        if (t > 0 && table[t].max_dim <= table[t - 1].max_dim)
            return fail(GFECH_E_ARG, "blocking table entries must have increasing max_dim");
    }
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table.assign(table, table + count);
    return GFECH_OK;
}

gfech_status gfech_echelonise_gf2(const uint64_t* A, int64_t m, int64_t n, int64_t ldw, const gfech_opts* opts,
                                  gfech_result** out) {
    return echelonise_gf2_impl(A, false, m, n, ldw, opts, nullptr, out);
}

gfech_status gfech_echelonise_gf2_dev(const uint64_t* A_dev, int64_t m, int64_t n, int64_t ldw,
                                      const gfech_opts* opts, void* stream, gfech_result** out) {
    return echelonise_gf2_impl(A_dev, true, m, n, ldw, opts, stream, out);
}

gfech_status gfech_echelonise_batch(int64_t count, const gfech_problem* probs, int32_t inputs_on_device,
                                    const gfech_opts* opts, void* stream, gfech_result** outs,
                                    gfech_status* per_problem) {
    if (count < 0 || (count > 0 && (!probs || !outs))) return fail(GFECH_E_ARG, "bad batch arguments");
    if (check_variant(opts)) return GFECH_E_ARG;
    gfech_status first = GFECH_OK;
    std::vector<int64_t> ok;
    for (int64_t t = 0; t < count; ++t) {
        outs[t] = nullptr;
        const gfech_problem& q = probs[t];
        gfech_status st = check_common(q.m, q.n, q.lda, q.p, q.A);
        if (!st && !inputs_on_device && !(opts && opts->skip_range_check)) {
            for (int64_t i = 0; i < q.m && !st; ++i)
                for (int64_t j = 0; j < q.n; ++j)
                    if (q.A[i * q.lda + j] >= q.p) { st = fail(GFECH_E_RANGE, "entry >= p"); break; }
        }
        if (per_problem) per_problem[t] = st;
        if (st) { if (!first) first = st; continue; }
        ok.push_back(t);
    }
    if (ok.empty()) return first;
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    std::vector<gfech::Problem> pv;
    std::vector<int64_t> run_idx;
    std::vector<void*> staged;
    // device inputs: one range check for all of them (one wait)
    std::vector<int64_t> bad(probs ? (size_t)count : 0, 0);
    if (inputs_on_device && !(opts && opts->skip_range_check)) {
        std::vector<gfech::Backend::RangeDesc> rd;
        std::vector<int64_t> who;
        for (int64_t t : ok) {
            const gfech_problem& q = probs[t];
            if (q.m <= 0 || q.n <= 0) continue;
            gfech::Backend::RangeDesc d;
            d.A = q.A; d.m = q.m; d.n = q.n; d.lda = q.lda; d.p = (int32_t)q.p;
            rd.push_back(d);
            who.push_back(t);
        }
        std::vector<int64_t> b;
        be->count_out_of_range_many(rd, b);
        for (size_t k = 0; k < who.size(); ++k) bad[(size_t)who[k]] = b[k];
    }
    for (int64_t t : ok) {
        const gfech_problem& q = probs[t];
        gfech::Problem pr;
        pr.m = q.m; pr.n = q.n; pr.lda = q.lda; pr.p = (int32_t)q.p; pr.A = q.A;
        pr.want = variant_of(opts);
        if (bad[(size_t)t]) {
            if (per_problem) per_problem[t] = bad[(size_t)t] > 0 ? GFECH_E_RANGE : GFECH_E_DEVICE;
            if (!first) first = fail(bad[(size_t)t] > 0 ? GFECH_E_RANGE : GFECH_E_DEVICE, "entry >= p");
            continue;
        }
        if (!inputs_on_device && q.m > 0 && q.n > 0) {
            void* d = be->alloc((size_t)(q.m * q.n));
            if (!d) { st = fail(GFECH_E_NOMEM, "staging allocation failed"); break; }
            std::vector<uint8_t> tmp((size_t)(q.m * q.n));
            for (int64_t i = 0; i < q.m; ++i) memcpy(tmp.data() + i * q.n, q.A + i * q.lda, (size_t)q.n);
            be->upload(d, tmp.data(), tmp.size());
            staged.push_back(d);
            pr.A = (const uint8_t*)d;
            pr.lda = q.n;
        }
        choose_blocks(pr.m, pr.n, opts, pr.row_blocks, pr.col_blocks);
        pv.push_back(pr);
        run_idx.push_back(t);
    }
    std::vector<gfech_result*> tmp_out(pv.size(), nullptr);
    if (!st && !pv.empty()) st = run(be, pv, tmp_out.data(), opts);
    for (void* d : staged) be->release(d);
    be->set_stream(nullptr);
    // map results back (problems that failed validation keep NULL)
    for (size_t k = 0; k < run_idx.size(); ++k) {
        outs[run_idx[k]] = tmp_out[k];
        if (per_problem) per_problem[run_idx[k]] = st;
    }
    if (st && !first) first = st;
    return first;
}

int64_t gfech_rank(const gfech_result* res) { return res ? res->r->r : -1; }

gfech_status gfech_shape(const gfech_result* res, int64_t* m, int64_t* n, uint32_t* p) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    if (m) *m = res->r->m;
    if (n) *n = res->r->n;
    if (p) *p = (uint32_t)res->r->p;
    return GFECH_OK;
}

gfech_status gfech_pivots(const gfech_result* res, int64_t* gamma, int64_t* rho) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    std::lock_guard<std::mutex> lk(R.be->lock());
    if (gamma) download_list(R.be, R.upsilon, R.r, gamma);
    if (rho) download_list(R.be, R.varrho, R.r, rho);
    return GFECH_OK;
}

gfech_status gfech_nonpivots(const gfech_result* res, int64_t* gamma_bar, int64_t* rho_bar) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    std::lock_guard<std::mutex> lk(R.be->lock());
    if (gamma_bar) download_list(R.be, R.upsilon_bar, R.n - R.r, gamma_bar);
    if (rho_bar) download_list(R.be, R.varrho_bar, R.m - R.r, rho_bar);
    return GFECH_OK;
}

gfech_status gfech_get_R(const gfech_result* res, uint8_t* R_, int64_t ldr) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_R(R)) return fail(GFECH_E_STATE, "the result was computed without R");
    if (R.r > 0 && R.n - R.r > 0 && (!R_ || ldr < R.n - R.r)) return fail(GFECH_E_ARG, "bad R buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    return download_matrix(R.be, R.Pfinal + R.offR, R.ldP, R.r, R.n - R.r, R_, ldr);
}

gfech_status gfech_get_M(const gfech_result* res, uint8_t* M, int64_t ldm) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_T(R)) return fail(GFECH_E_STATE, "the result was computed without the transformation");
    if (R.r > 0 && (!M || ldm < R.r)) return fail(GFECH_E_ARG, "bad M buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    return download_matrix(R.be, R.Pfinal + R.offM, R.ldP, R.r, R.r, M, ldm);
}

gfech_status gfech_get_K(const gfech_result* res, uint8_t* K, int64_t ldk) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_T(R)) return fail(GFECH_E_STATE, "the result was computed without the transformation");
    if (R.r > 0 && R.m - R.r > 0 && (!K || ldk < R.r)) return fail(GFECH_E_ARG, "bad K buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    return download_matrix(R.be, R.Kfinal, R.ldK, R.m - R.r, R.r, K, ldk);
}

gfech_status gfech_expand_rref_dev(const gfech_result* res, uint8_t* E, int64_t lde, void* stream) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_R(R)) return fail(GFECH_E_STATE, "the result was computed without R");
    if (R.r > 0 && R.n > 0 && (!E || lde < R.n)) return fail(GFECH_E_ARG, "bad E buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    R.be->set_stream(stream);
    expand_rref_ops(R, E, lde, R.be);
    R.be->sync();
    R.be->set_stream(nullptr);
    return R.be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_expand_transform_dev(const gfech_result* res, uint8_t* T, int64_t ldt, void* stream) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_T(R)) return fail(GFECH_E_STATE, "the result was computed without the transformation");
    if (R.m > 0 && (!T || ldt < R.m)) return fail(GFECH_E_ARG, "bad T buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    R.be->set_stream(stream);
    expand_transform_ops(R, T, ldt, R.be);
    R.be->sync();
    R.be->set_stream(nullptr);
    return R.be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_expand_rref(const gfech_result* res, uint8_t* E, int64_t lde) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_R(R)) return fail(GFECH_E_STATE, "the result was computed without R");
    if (R.r == 0 || R.n == 0) return GFECH_OK;
    if (!E || lde < R.n) return fail(GFECH_E_ARG, "bad E buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    uint8_t* d = (uint8_t*)R.be->alloc((size_t)(R.r * R.n));
    if (!d) return fail(GFECH_E_NOMEM, "device allocation failed");
    expand_rref_ops(R, d, R.n, R.be);
    download_matrix(R.be, d, R.n, R.r, R.n, E, lde);
    R.be->release(d);
    return R.be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_expand_transform(const gfech_result* res, uint8_t* T, int64_t ldt) {
    if (!res) return fail(GFECH_E_ARG, "NULL result");
    const gfech::Result& R = *res->r;
    if (!has_T(R)) return fail(GFECH_E_STATE, "the result was computed without the transformation");
    if (R.m == 0) return GFECH_OK;
    if (!T || ldt < R.m) return fail(GFECH_E_ARG, "bad T buffer");
    std::lock_guard<std::mutex> lk(R.be->lock());
    uint8_t* d = (uint8_t*)R.be->alloc((size_t)(R.m * R.m));
    if (!d) return fail(GFECH_E_NOMEM, "device allocation failed");
    expand_transform_ops(R, d, R.m, R.be);
    download_matrix(R.be, d, R.m, R.m, R.m, T, ldt);
    R.be->release(d);
    return R.be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_device_view(const gfech_result* res, gfech_view* v) {
    if (!res || !v) return fail(GFECH_E_ARG, "NULL argument");
    const gfech::Result& R = *res->r;
    v->R = has_R(R) ? R.Pfinal + R.offR : nullptr; v->ldr = R.ldP;
    v->M = has_T(R) ? R.Pfinal + R.offM : nullptr; v->ldm = R.ldP;
    v->K = has_T(R) ? R.Kfinal : nullptr; v->ldk = R.ldK;
    v->gamma = R.upsilon; v->gamma_bar = R.upsilon_bar;
    v->rho = R.varrho; v->rho_bar = R.varrho_bar;
    return GFECH_OK;
}

gfech_status gfech_get_stats(const gfech_result* res, gfech_stats* s) {
    if (!res || !s) return fail(GFECH_E_ARG, "NULL argument");
    const gfech::Stats& t = res->r->stats;
    s->mac_cleardown = t.cd_mad;
    s->mac_ech = t.ech;
    s->mac_updaterow = t.ur_mad;
    s->mac_trafo = t.urt_mad;
    s->mac_clearup = t.cu_mad;
    s->gather_bytes = t.gather_bytes;
    s->layers = t.layers;
    s->echs = t.echs;
    s->gemms = t.gemms;
    s->launches = t.launches;
    s->syncs = t.syncs;
    s->block_rows = (int64_t)res->r->row_blocks.size();
    s->block_cols = (int64_t)res->r->col_blocks.size();
    s->ms_mad = t.kernel_ms[0];
    s->ms_ech = t.kernel_ms[1];
    s->ms_small = t.kernel_ms[2];
    s->launches_mad = t.kernel_launches[0];
    s->launches_ech = t.kernel_launches[1];
    s->launches_small = t.kernel_launches[2];
    s->mad_bytes = t.mad_bytes;
    s->mac_mad_timed = t.kernel_mac[0];
    s->variant = res->r->want;
    s->tail_checks = t.tail_checks;
    s->ech_reruns = t.ech_reruns;
    return GFECH_OK;
}

void gfech_result_free(gfech_result* res) {
    // the result's work is complete; releasing its memory takes only the
    // backend's memory-cache lock, so this never waits for an engine iteration
    delete res;
}

static gfech_status mad_check(const gfech_mad_desc& d) {
    if (d.M < 0 || d.N < 0 || d.K < 0) return fail(GFECH_E_ARG, "negative MAD size");
    if (d.M > INT32_MAX || d.N > INT32_MAX || d.K > 65536) return fail(GFECH_E_TOO_BIG, "MAD size too large");
    if (d.p > 251 || !is_prime(d.p)) return fail(GFECH_E_FIELD, "p must be a prime <= 251");
    if (d.M == 0 || d.N == 0) return GFECH_OK;
    if (!d.D || d.ldd < d.N) return fail(GFECH_E_ARG, "bad D");
    if (d.K > 0 && (!d.A || !d.B || d.lda < d.K || d.ldb < d.N)) return fail(GFECH_E_ARG, "bad A or B");
    if (d.C && d.ldc < d.N) return fail(GFECH_E_ARG, "bad C");
    return GFECH_OK;
}

static gfech::GemmDesc to_gemm(const gfech_mad_desc& d) {
    gfech::GemmDesc g;
    g.M = (int32_t)d.M; g.N = (int32_t)d.N; g.K = (int32_t)d.K; g.p = (int32_t)d.p;
    g.A = d.A; g.lda = d.lda; g.B = d.B; g.ldb = d.ldb; g.brow = d.brow;
    g.C = d.C; g.ldc = d.ldc; g.crow = d.crow; g.D = d.D; g.ldd = d.ldd;
    return g;
}

static gfech_status mad_batch(int64_t count, const gfech_mad_desc* descs, void* stream, double* kernel_ms) {
    if (count < 0 || (count > 0 && !descs)) return fail(GFECH_E_ARG, "bad MAD batch");
    std::vector<gfech::GemmDesc> gs;
    for (int64_t t = 0; t < count; ++t) {
        gfech_status st = mad_check(descs[t]);
        if (st) return st;
        if (descs[t].M && descs[t].N) gs.push_back(to_gemm(descs[t]));
    }
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    if (kernel_ms) {
        be->take_profile();                 // drop events of earlier work
        be->set_profile(2);                 // MAD launches carry start and stop events
    }
    if (!gs.empty()) be->gemm(gs);
    be->sync();
    if (kernel_ms) {
        *kernel_ms = be->take_profile().ms[0];
        be->set_profile(0);
    }
    be->set_stream(nullptr);
    return be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_mad_batch_dev(int64_t count, const gfech_mad_desc* descs, void* stream) {
    return mad_batch(count, descs, stream, nullptr);
}

gfech_status gfech_mad_batch_dev_timed(int64_t count, const gfech_mad_desc* descs, void* stream,
                                       double* kernel_ms) {
    if (!kernel_ms) return fail(GFECH_E_ARG, "kernel_ms is NULL");
    *kernel_ms = 0;
    return mad_batch(count, descs, stream, kernel_ms);
}

gfech_status gfech_mad_dev(int64_t M, int64_t N, int64_t K, uint32_t p, const uint8_t* A, int64_t lda,
                           const uint8_t* B, int64_t ldb, const int32_t* brow, const uint8_t* C, int64_t ldc,
                           const int32_t* crow, uint8_t* D, int64_t ldd, void* stream) {
    gfech_mad_desc d;
    memset(&d, 0, sizeof(d));
    d.M = M; d.N = N; d.K = K; d.p = p;
    d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.brow = brow;
    d.C = C; d.ldc = ldc; d.crow = crow; d.D = D; d.ldd = ldd;
    return gfech_mad_batch_dev(1, &d, stream);
}

gfech_status gfech_mad_gf2_dev(int64_t M, int64_t N, int64_t K, const uint64_t* A, int64_t lda, const uint64_t* B,
                               int64_t ldb, const uint64_t* C, int64_t ldc, uint64_t* D, int64_t ldd, void* stream) {
    if (M < 0 || N < 0 || K < 0) return fail(GFECH_E_ARG, "negative size");
    if (M == 0 || N == 0) return GFECH_OK;
    const int64_t wn = (N + 63) / 64, wk = (K + 63) / 64;
    if (!D || ldd < wn || (K > 0 && (!A || !B || lda < wk || ldb < wn)) || (C && ldc < wn))
        return fail(GFECH_E_ARG, "bad GF(2) MAD buffers");
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    gfech::Gf2MadDesc d;
    d.M = M; d.N = N; d.K = K;
    d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = ldc; d.D = D; d.ldd = ldd;
    be->mad_gf2(d);
    be->sync();
    be->set_stream(nullptr);
    return be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

gfech_status gfech_ech_dev(const uint8_t* H, int64_t rows, int64_t cols, int64_t ldh, uint32_t p, int32_t* prow,
                           int32_t* qrow, int32_t* pcol, int32_t* qcol, uint8_t* M, int64_t ldm, uint8_t* K,
                           int64_t ldk, uint8_t* R, int64_t ldr, int64_t* rank, void* stream) {
    if (!rank) return fail(GFECH_E_ARG, "rank is NULL");
    *rank = 0;
    if (rows < 0 || cols < 0) return fail(GFECH_E_ARG, "negative size");
    if (rows + cols > 8192) return fail(GFECH_E_TOO_BIG, "block too large for one ECH");
    if (p > 251 || !is_prime(p)) return fail(GFECH_E_FIELD, "p must be a prime <= 251");
    if (rows == 0 || cols == 0) return GFECH_OK;
    int64_t mr = rows < cols ? rows : cols;
    if (!H || ldh < cols || !prow || !qrow || !pcol || !qcol || !M || !K || !R || ldm < mr || ldk < mr ||
        ldr < cols)
        return fail(GFECH_E_ARG, "bad ECH buffers");
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    be->set_stream(stream);
    int64_t ldw = cols + mr;
    uint8_t* work = (uint8_t*)be->alloc((size_t)(rows * ldw));
    int32_t* cnt = (int32_t*)be->alloc(sizeof(int32_t));
    if (!work || !cnt) {
        be->release(work);
        be->release(cnt);
        be->set_stream(nullptr);
        return fail(GFECH_E_NOMEM, "ECH workspace");
    }
    gfech::EchDesc e;
    e.rows = (int32_t)rows; e.cols = (int32_t)cols; e.p = (int32_t)p;
    e.H = H; e.ldh = ldh; e.work = work; e.ldw = ldw; e.rcount = cnt;
    e.prow = prow; e.qrow = qrow; e.pcol = pcol; e.qcol = qcol;
    e.Mo = M; e.ldm = ldm; e.Ko = K; e.ldk = ldk; e.Ro = R; e.ldr = ldr;
    be->ech({e});
    int32_t r = 0;
    be->download(&r, cnt, sizeof(int32_t));
    be->release(work);
    be->release(cnt);
    be->set_stream(nullptr);
    *rank = r;
    return be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

static_assert(GFECH_NOALLOC_SCRATCH_BYTES == (int64_t)gfech::kFixedScratchBytes, "fixed workspace size");

gfech_status gfech_ech_dev_noalloc(const uint8_t* H, int64_t rows, int64_t cols, int64_t ldh, uint32_t p,
                                   int32_t* prow, int32_t* qrow, int32_t* pcol, int32_t* qcol, uint8_t* M,
                                   int64_t ldm, uint8_t* K, int64_t ldk, uint8_t* R, int64_t ldr, int32_t* rank_dev,
                                   void* stream) {
    if (!rank_dev) return fail(GFECH_E_ARG, "rank_dev is NULL");
    if (rows < 0 || cols < 0) return fail(GFECH_E_ARG, "negative size");
    if (rows + cols > 8192) return fail(GFECH_E_TOO_BIG, "block too large for one ECH");
    if (p > 251 || !is_prime(p)) return fail(GFECH_E_FIELD, "p must be a prime <= 251");
    const int64_t mr = rows < cols ? rows : cols;
    const int64_t ldw = cols + mr;
    if (rows > 0 && cols > 0 &&
        (!H || ldh < cols || !prow || !qrow || !pcol || !qcol || !M || !K || !R || ldm < mr || ldk < mr || ldr < cols))
        return fail(GFECH_E_ARG, "bad ECH buffers");
    if ((size_t)(rows * ldw) > gfech::kFixedScratchBytes)
        return fail(GFECH_E_TOO_BIG, "the block's workspace exceeds the fixed workspace");
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    if (!be) return st;
    std::lock_guard<std::mutex> lk(be->lock());
    uint8_t* ws = be->fixed_scratch();
    if (!ws) return fail(GFECH_E_DEVICE, "no fixed workspace on this device");
    be->set_stream(stream);
    if (rows == 0 || cols == 0) {
        // rank 0, written by a kernel (no memset, no copy)
        gfech::FillDesc f;
        f.rows = 1; f.cols = (int32_t)sizeof(int32_t); f.dst = (uint8_t*)rank_dev; f.ldd = sizeof(int32_t);
        be->fill({f});
    } else {
        gfech::EchDesc e;
        e.rows = (int32_t)rows; e.cols = (int32_t)cols; e.p = (int32_t)p;
        e.H = H; e.ldh = ldh; e.work = ws; e.ldw = ldw; e.rcount = rank_dev;
        e.prow = prow; e.qrow = qrow; e.pcol = pcol; e.qcol = qcol;
        e.Mo = M; e.ldm = ldm; e.Ko = K; e.ldk = ldk; e.Ro = R; e.ldr = ldr;
        be->ech({e});
    }
    be->set_stream(nullptr);
    return be->error() ? fail(GFECH_E_DEVICE, "device error") : GFECH_OK;
}

// ---------------------------------------------------------------- serving

// Requests are sorted into size classes by max(m, n).  Each class has its own
// engine, its own backend instance (streams, lanes, memory cache, lock) and
// its own worker thread: a class's requests share launches (continuous
// batching), and the phases of a large problem never hold back the small
// ones, whose iterations are short and whose work runs on other streams.
// Admission is first come first served within a class, against one
// device-memory budget shared by the classes.  Inputs are copied by a
// backend instance of their own (its lock is held only for the copy or a
// release), so a submission never waits for an engine iteration.  Lock
// order: a class backend's lock, then the input backend's lock, then the
// server's mu; never the reverse.
struct gfech_server {
    struct Req {
        uint64_t ticket = 0;
        gfech::Problem pr;
        uint8_t* input = nullptr;     // device copy (input backend), owned until the request finishes
        size_t footprint = 0;
    };
    struct Class {
        int64_t max_dim = 0;                  // largest max(m, n) of the class; 0 = no limit
        gfech::Backend* be = nullptr;
        void* stream = nullptr;               // lane 0 of the class's engine
        std::unique_ptr<gfech::Engine> eng;   // used with be->lock() held
        std::deque<Req> queue;                // under mu
        std::map<int64_t, Req> running;       // engine id -> request, under mu
        std::vector<uint64_t> cancels;        // tickets of running requests to cancel, under mu
        std::condition_variable work;
        std::thread worker;
    };
    std::vector<std::unique_ptr<Class>> classes;
    gfech::Backend* in_be = nullptr;  // the input copies: allocated, copied and released with its lock
    void* in_stream = nullptr;
    size_t budget = 0;
    int32_t max_active = 0;
    std::mutex mu;                    // everything marked "under mu" and the fields below
    std::condition_variable done;
    std::map<uint64_t, std::pair<gfech_status, gfech_result*>> finished;
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t bytes_in_flight = 0;       // footprints of the admitted requests of every class
    int64_t active = 0;
    gfech_server_stats counters{};

    Class& class_of(int64_t m, int64_t n) {
        const int64_t d = std::max(m, n);
        for (auto& k : classes)
            if (k->max_dim == 0 || d <= k->max_dim) return *k;
        return *classes.back();
    }
    // under mu: the class's next request may be admitted now
    bool admissible(const Class& k) const {
        return !k.queue.empty() && (max_active <= 0 || active < max_active) &&
               (bytes_in_flight == 0 || bytes_in_flight + k.queue.front().footprint <= budget);
    }
    bool known(uint64_t ticket) const {
        if (finished.count(ticket)) return true;
        for (auto& k : classes) {
            for (auto& r : k->queue) if (r.ticket == ticket) return true;
            for (auto& kv : k->running) if (kv.second.ticket == ticket) return true;
        }
        return false;
    }

    // the engine's work on the input is complete (it synchronises when a
    // problem finishes or fails)
    void release_input(uint8_t* input) {
        if (!input) return;
        std::lock_guard<std::mutex> lk(in_be->lock());
        in_be->release(input);
    }

    // admit what fits, advance the class's active problems by one phase, hand
    // out the finished ones
    void iterate(Class& k) {
        std::lock_guard<std::mutex> lk(k.be->lock());
        k.be->set_stream(k.stream);
        std::vector<uint8_t*> spent;          // inputs to release (after mu is released)
        {
            std::lock_guard<std::mutex> q(mu);
            while (admissible(k)) {
                Req r = k.queue.front();
                int st = 0;
                const int64_t id = k.eng->add(r.pr, &st);
                if (id < 0) {
                    if (k.eng->active() > 0) break;            // wait until memory frees up
                    k.queue.pop_front();
                    spent.push_back(r.input);
                    finished[r.ticket] = {GFECH_E_NOMEM, nullptr};
                    done.notify_all();
                    continue;
                }
                k.queue.pop_front();
                k.running[id] = r;
                bytes_in_flight += r.footprint;
                active++;
                counters.admitted++;
            }
            counters.peak_bytes_in_flight = std::max<int64_t>(counters.peak_bytes_in_flight, (int64_t)bytes_in_flight);
            counters.peak_active = std::max<int64_t>(counters.peak_active, active);
            for (uint64_t t : k.cancels)
                for (auto& kv : k.running)
                    if (kv.second.ticket == t) k.eng->cancel(kv.first);
            k.cancels.clear();
        }
        for (uint8_t* in : spent) release_input(in);
        spent.clear();
        if (k.eng->active()) k.eng->step();
        std::vector<gfech::Engine::Done> fin = k.eng->take_done();
        if (!fin.empty()) {
            std::lock_guard<std::mutex> q(mu);
            for (auto& d : fin) {
                auto it = k.running.find(d.id);
                if (it == k.running.end()) continue;
                spent.push_back(it->second.input);
                gfech_result* res = nullptr;
                if (d.result) {
                    res = new gfech_result();
                    res->r = std::move(d.result);
                }
                finished[it->second.ticket] = {status_of(d.status), res};
                bytes_in_flight -= it->second.footprint;
                active--;
                counters.finished++;
                k.running.erase(it);
            }
            done.notify_all();
            for (auto& o : classes) o->work.notify_all();     // memory freed: other classes may admit
        }
        for (uint8_t* in : spent) release_input(in);
        k.be->set_stream(nullptr);
    }

    void loop(Class& k) {
        for (;;) {
            {
                std::unique_lock<std::mutex> q(mu);
                k.work.wait(q, [&] { return stop || admissible(k) || !k.running.empty(); });
                if (stop && k.running.empty()) break;
            }
            iterate(k);
        }
    }
};

gfech_status gfech_server_create(const gfech_server_cfg* cfg, gfech_server** out) {
    if (!out) return fail(GFECH_E_ARG, "out is NULL");
    *out = nullptr;
    const int32_t nclass = cfg && cfg->size_classes > 0 ? cfg->size_classes : 3;
    if (nclass > 3) return fail(GFECH_E_ARG, "at most 3 size classes");
    // class limits on max(m, n): one block; one block column; the rest
    static const int64_t kLimits[3] = {512, 2048, 0};
    std::unique_ptr<gfech_server> s(new gfech_server());
    {
        std::string err;
        s->in_be = gfech::backend_acquire(&err);
        if (!s->in_be) return fail(GFECH_E_DEVICE, err.empty() ? "no device backend" : err);
        std::lock_guard<std::mutex> lk(s->in_be->lock());
        s->in_stream = s->in_be->create_stream();
    }
    for (int32_t c = 0; c < nclass; ++c) {
        std::unique_ptr<gfech_server::Class> k(new gfech_server::Class());
        k->max_dim = c == nclass - 1 ? 0 : kLimits[c];
        std::string err;
        k->be = gfech::backend_acquire(&err);
        if (!k->be) {
            for (auto& o : s->classes) gfech::backend_release(o->be);
            gfech::backend_release(s->in_be);
            return fail(GFECH_E_DEVICE, err.empty() ? "no device backend" : err);
        }
        std::lock_guard<std::mutex> lk(k->be->lock());
        k->stream = k->be->create_stream();
        k->eng.reset(new gfech::Engine(*k->be));
        s->classes.push_back(std::move(k));
    }
    s->budget = (cfg && cfg->hbm_budget_bytes > 0) ? (size_t)cfg->hbm_budget_bytes : ((size_t)200 << 30);
    s->max_active = cfg ? cfg->max_active : 0;
    gfech_server* raw = s.get();
    for (auto& k : s->classes) {
        gfech_server::Class* kp = k.get();
        k->worker = std::thread([raw, kp] { raw->loop(*kp); });
    }
    *out = s.release();
    return GFECH_OK;
}

gfech_status gfech_server_submit(gfech_server* s, const gfech_problem* prob, int32_t input_on_device,
                                 uint64_t* ticket) {
    if (!s || !prob || !ticket) return fail(GFECH_E_ARG, "null argument");
    *ticket = 0;
    const int64_t m = prob->m, n = prob->n, lda = prob->lda;
    const uint32_t p = prob->p;
    gfech_status st = check_common(m, n, lda, p, prob->A);
    if (st) return st;
    if (!input_on_device) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (prob->A[i * lda + j] >= p) return fail(GFECH_E_RANGE, "entry >= p");
    }
    gfech_server::Class& k = s->class_of(m, n);
    gfech_server::Req r;
    r.pr.m = m;
    r.pr.n = n;
    r.pr.lda = std::max<int64_t>(n, 1);
    r.pr.p = (int32_t)p;
    choose_blocks(m, n, nullptr, r.pr.row_blocks, r.pr.col_blocks);
    r.footprint = k.eng->footprint(r.pr);    // sizes only: no device work
    if (r.footprint > s->budget) return fail(GFECH_E_TOO_BIG, "the problem alone exceeds the memory budget");
    {
        // the input is checked and copied by the input backend on its stream,
        // complete on return (the caller may reuse its buffer); nothing waits
        // for an engine
        gfech::Backend* be = s->in_be;
        std::lock_guard<std::mutex> lk(be->lock());
        be->set_stream(s->in_stream);
        if (input_on_device && m > 0 && n > 0) {
            const int64_t bad = be->count_out_of_range(prob->A, m, n, lda, (int32_t)p);
            if (bad != 0) {
                be->set_stream(nullptr);
                return fail(bad > 0 ? GFECH_E_RANGE : GFECH_E_DEVICE, bad > 0 ? "entry >= p" : "device error");
            }
        }
        // the request owns a packed device copy of its input
        if (m > 0 && n > 0) {
            r.input = (uint8_t*)be->alloc((size_t)(m * n));
            if (!r.input) {
                be->set_stream(nullptr);
                return fail(GFECH_E_NOMEM, "device allocation of the input failed");
            }
            if (input_on_device && lda == n) {
                be->copy(r.input, prob->A, (size_t)(m * n));
            } else if (input_on_device) {
                for (int64_t i = 0; i < m; ++i) be->copy(r.input + i * n, prob->A + i * lda, (size_t)n);
            } else if (lda == n) {
                be->upload(r.input, prob->A, (size_t)(m * n));
            } else {
                std::vector<uint8_t> tmp((size_t)(m * n));
                for (int64_t i = 0; i < m; ++i) memcpy(tmp.data() + i * n, prob->A + i * lda, (size_t)n);
                be->upload(r.input, tmp.data(), (size_t)(m * n));
            }
            be->sync_lane0();
        }
        be->set_stream(nullptr);
        r.pr.A = r.input;
    }
    {
        std::lock_guard<std::mutex> q(s->mu);
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        k.queue.push_back(r);
    }
    k.work.notify_all();
    return GFECH_OK;
}

namespace {
// with s->mu held: the outcome of a ticket, if there is one
gfech_status take_finished(gfech_server* s, uint64_t ticket, gfech_result** out, bool* known) {
    auto it = s->finished.find(ticket);
    if (it != s->finished.end()) {
        const gfech_status st = it->second.first;
        *out = it->second.second;
        s->finished.erase(it);
        *known = true;
        return st == GFECH_OK ? GFECH_OK : fail(st, "request failed");
    }
    *known = s->known(ticket);
    return GFECH_OK;
}
}  // namespace

gfech_status gfech_server_poll(gfech_server* s, uint64_t ticket, gfech_result** out) {
    if (!s || !out) return fail(GFECH_E_ARG, "null argument");
    *out = nullptr;
    std::lock_guard<std::mutex> q(s->mu);
    bool known = false;
    gfech_status st = take_finished(s, ticket, out, &known);
    if (!known) return fail(GFECH_E_ARG, "unknown ticket");
    return st;
}

gfech_status gfech_server_cancel(gfech_server* s, uint64_t ticket) {
    if (!s) return fail(GFECH_E_ARG, "null argument");
    gfech_server::Req dropped;
    {
        std::lock_guard<std::mutex> q(s->mu);
        if (!s->known(ticket)) return fail(GFECH_E_ARG, "unknown ticket");
        for (auto& k : s->classes) {
            for (auto it = k->queue.begin(); it != k->queue.end(); ++it) {
                if (it->ticket != ticket) continue;
                dropped = *it;
                k->queue.erase(it);
                s->finished[ticket] = {GFECH_E_CANCELLED, nullptr};
                break;
            }
            for (auto& kv : k->running)
                if (kv.second.ticket == ticket) k->cancels.push_back(ticket);
        }
    }
    // its input was copied completely when it was submitted
    s->release_input(dropped.input);
    s->done.notify_all();
    for (auto& k : s->classes) k->work.notify_all();
    return GFECH_OK;
}

gfech_status gfech_server_get_stats(gfech_server* s, gfech_server_stats* stats) {
    if (!s || !stats) return fail(GFECH_E_ARG, "null argument");
    std::lock_guard<std::mutex> q(s->mu);
    *stats = s->counters;
    return GFECH_OK;
}

gfech_status gfech_server_wait(gfech_server* s, uint64_t ticket, gfech_result** out) {
    if (!s || !out) return fail(GFECH_E_ARG, "null argument");
    *out = nullptr;
    std::unique_lock<std::mutex> q(s->mu);
    for (;;) {
        bool known = false;
        gfech_status st = take_finished(s, ticket, out, &known);
        if (!known) return fail(GFECH_E_ARG, "unknown ticket");
        if (*out || st != GFECH_OK) return st;
        s->done.wait(q);
    }
}

void gfech_server_destroy(gfech_server* s) {
    if (!s) return;
    // queued requests are dropped, running ones finish
    std::vector<std::deque<gfech_server::Req>> dropped(s->classes.size());
    {
        std::lock_guard<std::mutex> q(s->mu);
        s->stop = true;
        for (size_t c = 0; c < s->classes.size(); ++c) dropped[c].swap(s->classes[c]->queue);
    }
    // their inputs were copied completely when they were submitted
    for (auto& q : dropped)
        for (auto& r : q) s->release_input(r.input);
    for (auto& k : s->classes) k->work.notify_all();
    for (auto& k : s->classes)
        if (k->worker.joinable()) k->worker.join();
    std::vector<gfech_result*> unclaimed;
    {
        std::lock_guard<std::mutex> q(s->mu);
        for (auto& kv : s->finished) if (kv.second.second) unclaimed.push_back(kv.second.second);
        s->finished.clear();
    }
    for (gfech_result* r : unclaimed) gfech_result_free(r);
    for (auto& k : s->classes) {
        {
            std::lock_guard<std::mutex> lk(k->be->lock());
            k->eng.reset();
            k->be->destroy_stream(k->stream);
        }
        // the backend instance goes back to the pool (results of this server
        // still refer to it)
        gfech::backend_release(k->be);
    }
    {
        std::lock_guard<std::mutex> lk(s->in_be->lock());
        s->in_be->destroy_stream(s->in_stream);
    }
    gfech::backend_release(s->in_be);
    delete s;
}

const char* gfech_strerror(gfech_status s) {
    switch (s) {
        case GFECH_OK: return "ok";
        case GFECH_E_ARG: return "invalid argument";
        case GFECH_E_FIELD: return "p is not a prime <= 251";
        case GFECH_E_RANGE: return "input entry >= p";
        case GFECH_E_NOMEM: return "out of memory";
        case GFECH_E_TOO_BIG: return "problem too large";
        case GFECH_E_DEVICE: return "device error";
        case GFECH_E_CANCELLED: return "cancelled";
        case GFECH_E_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* gfech_last_error(void) { return g_last_error.c_str(); }

const char* gfech_backend_name(void) {
    gfech_status st = GFECH_OK;
    gfech::Backend* be = get_backend(&st);
    return be ? be->name() : "unavailable";
}

}  // extern "C"
