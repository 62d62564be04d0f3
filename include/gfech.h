/*
 * gfech: blocked Gaussian elimination over a prime field GF(p), p <= 251, on
 * an MI355X (gfx950) GPU.  C ABI of libgfech.so.
 *
 * The method is that of Linton, Nebe, Niemeyer, Parker and Thackray, "A
 * parallel algorithm for Gaussian elimination over finite fields" (arXiv
 * 1806.04211).  For A in GF(p)^{m x n} of rank r the library computes, as in
 * Eq. (2) of Section 3.1 (the whole-matrix form of Remark 2.3, Eq. (1)),
 *
 *     [[M, 0], [K, 1]] * [rho; rho_bar] * A * [gamma^tr  gamma_bar^tr]
 *         = [[-1, R], [0, 0]]
 *
 * with rho the selected rows (r of them), gamma the pivot columns, M (r x r),
 * K ((m - r) x r) and R (r x (n - r)): the *negative* reduced echelon form the
 * paper uses.  Pivot rule (Section 1): a row's pivot is its first non-zero
 * entry and rows are taken in their original order, so row i is selected
 * exactly when it is outside the span of rows 0..i-1; with that rule every
 * output is unique.  The standard forms are available too: the RREF
 * E = [1 | -R] * P_gamma^-1 (pivots +1) and T = [[-M, 0], [K, 1]] * P_rho with
 * T * A = [E; 0] (T = A^-1 when A is invertible).
 *
 * Conventions of every call:
 *   - sizes and leading dimensions are int64_t counts of elements;
 *   - matrices are row-major with an explicit leading dimension (>= columns);
 *   - field elements are canonical residues in [0, p), one per uint8_t;
 *   - index lists are 0-based and ascending;
 *   - rows of M and R are ordered by pivot column, columns of M and K by
 *     selected row, rows of K by non-selected row, columns of R ascending.
 * Every call returns a status; nothing aborts or throws across the ABI.
 * Calls are serialised inside the library (one device per process).
 */
#ifndef GFECH_H
#define GFECH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gfech_status {
    GFECH_OK = 0,
    GFECH_E_ARG = 1,        /* null pointer, negative size, leading dimension too small */
    GFECH_E_FIELD = 2,      /* p is not a prime <= 251 */
    GFECH_E_RANGE = 3,      /* an input entry is >= p (inputs are never reduced silently) */
    GFECH_E_NOMEM = 4,      /* device or host allocation failed */
    GFECH_E_TOO_BIG = 5,    /* a size exceeds what the kernels index (2^31 - 1 per dimension) */
    GFECH_E_DEVICE = 6,     /* HIP runtime error or no usable gfx950 device */
    GFECH_E_CANCELLED = 7,  /* stopped by the watchdog (opts.timeout_ms) or gfech_server_cancel */
    GFECH_E_STATE = 8       /* call not valid for this object */
} gfech_status;

/* What a call computes: the variants of Gaussian elimination the paper's
 * introduction (Section 1) lists, each a subset of the full result.
 *   GFECH_WANT_RREF_T  the reduced echelon form with the transformation: rank,
 *                      gamma, rho, R, M, K (the default; everything below);
 *   GFECH_WANT_RREF    the reduced echelon form without the transformation:
 *                      rank, gamma, rho and R (E); the UpdateRowTrafo products
 *                      of Step 1 and the M part of Step 3 are not run, and
 *                      M, K and T are not available (GFECH_E_STATE);
 *   GFECH_WANT_RANK    the rank with the pivot columns gamma and the selected
 *                      rows rho: additionally Step 3 is not run and R and E
 *                      are not available either.
 * Every output that a variant provides equals the full result's. */
enum { GFECH_WANT_RREF_T = 0, GFECH_WANT_RREF = 1, GFECH_WANT_RANK = 2 };

/* Options.  Zero-initialised options (or NULL) select the defaults. */
typedef struct gfech_opts {
    int64_t block_rows;     /* a_i target (Section 3.1); 0 = automatic */
    int64_t block_cols;     /* b_j target; 0 = automatic */
    int32_t skip_range_check; /* 1: the caller guarantees entries < p (no validation pass) */
    int32_t profile;        /* 1: time every kernel launch with device events, 2: only the MAD
                               launches, 3: a pseudo-random quarter of the MAD launches
                               (see gfech_stats);
                               0: no events */
    int32_t variant;        /* GFECH_WANT_*; other values give GFECH_E_ARG */
    int32_t timeout_ms;     /* > 0: a watchdog.  A call still running after this many
                               milliseconds stops at its next phase boundary (a layer of
                               Step 1 or a launch of Step 3), frees what it holds and
                               returns GFECH_E_CANCELLED; 0: no limit */
    int32_t reserved[4];
} gfech_opts;

/* Block sizes (Section 3.1) chosen by measurement: when a call's options
 * leave block_rows and block_cols at 0, the first entry with
 * max(m, n) <= max_dim gives them (0 in one of them: the same as the other);
 * problems above every entry, or with no table installed, get the built-in
 * choice (one block up to 512 x 512, else blocks of 256 rows and 2048
 * columns).  Block sizes never change results.  gfech_set_blocking copies
 * the table (entries with strictly increasing max_dim) and replaces the
 * previous one; count 0 removes it.  The package's tuner writes such tables. */
typedef struct gfech_blocking {
    int64_t max_dim;
    int64_t block_rows, block_cols;
} gfech_blocking;
gfech_status gfech_set_blocking(const gfech_blocking* table, int64_t count);

/* Opaque, library-owned result; immutable once returned.  Its matrices stay
 * in device memory (HBM) until copied out by the getters below. */
typedef struct gfech_result gfech_result;

/* Echelonise A (host memory, m x n, leading dimension lda) over GF(p).
 * m = 0 or n = 0 is valid (rank 0).  A is only read during the call.
 * On success *out owns a new result; on failure *out is NULL. */
gfech_status gfech_echelonise_u8(const uint8_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p,
                                 const gfech_opts* opts, gfech_result** out);

/* Same with A in device memory (a HIP device pointer).  `stream` is a
 * hipStream_t (NULL = the default stream); the call returns after the work on
 * that stream has completed.  The result stays in device memory. */
gfech_status gfech_echelonise_u8_dev(const uint8_t* A_dev, int64_t m, int64_t n, int64_t lda, uint32_t p,
                                     const gfech_opts* opts, void* stream, gfech_result** out);

/* GF(2) with bit-packed rows (the field of the paper's largest runs,
 * Section 6): bit b of word w of row i is entry (i, 64 w + b), least
 * significant bit first; each row has ldw >= ceil(n / 64) words.  Bits past
 * column n - 1 in a row's last word (pad bits) must be zero: a set pad bit
 * gives GFECH_E_RANGE (skip_range_check skips that check).  The result is
 * that of gfech_echelonise_u8 on the unpacked matrix with p = 2 (Eq. (2);
 * over GF(2), -1 = 1, so the paper's negative form and the standard form
 * coincide); the input is unpacked on the device, one byte per entry,
 * straight into the working panels of the elimination (no unpacked copy of
 * the input is made).  Host input, and device input ordered on `stream`. */
gfech_status gfech_echelonise_gf2(const uint64_t* A, int64_t m, int64_t n, int64_t ldw, const gfech_opts* opts,
                                  gfech_result** out);
gfech_status gfech_echelonise_gf2_dev(const uint64_t* A_dev, int64_t m, int64_t n, int64_t ldw,
                                      const gfech_opts* opts, void* stream, gfech_result** out);

/* One independent problem of a batch. */
typedef struct gfech_problem {
    const uint8_t* A;       /* host or device pointer, as the batch call says */
    int64_t m, n, lda;
    uint32_t p;
    uint32_t reserved;
} gfech_problem;

/* Echelonise `count` independent matrices together: every job of every
 * problem runs in shared grouped launches.  inputs_on_device selects whether
 * probs[t].A are device (1) or host (0) pointers.  outs[t] receives a result
 * or NULL; per_problem[t] (optional) its status.  Returns GFECH_OK when every
 * problem succeeded, else the first failing status. */
gfech_status gfech_echelonise_batch(int64_t count, const gfech_problem* probs, int32_t inputs_on_device,
                                    const gfech_opts* opts, void* stream, gfech_result** outs,
                                    gfech_status* per_problem);

/* Queries. */
int64_t gfech_rank(const gfech_result* res);                  /* r, or -1 for NULL */
gfech_status gfech_shape(const gfech_result* res, int64_t* m, int64_t* n, uint32_t* p);

/* gamma[r] pivot columns and rho[r] selected rows (host buffers, ascending). */
gfech_status gfech_pivots(const gfech_result* res, int64_t* gamma, int64_t* rho);
/* gamma_bar[n - r] non-pivot columns and rho_bar[m - r] non-selected rows. */
gfech_status gfech_nonpivots(const gfech_result* res, int64_t* gamma_bar, int64_t* rho_bar);

/* Copy the paper-form matrices into host buffers (row-major, given ld):
 * R is r x (n - r), M is r x r, K is (m - r) x r.  GFECH_E_STATE when the
 * result's variant does not include the matrix (and likewise for E, T and
 * the device view's pointers, which are then NULL). */
gfech_status gfech_get_R(const gfech_result* res, uint8_t* R, int64_t ldr);
gfech_status gfech_get_M(const gfech_result* res, uint8_t* M, int64_t ldm);
gfech_status gfech_get_K(const gfech_result* res, uint8_t* K, int64_t ldk);

/* Standard forms into host buffers: E is r x n (the RREF, pivots +1);
 * T is m x m with T * A = [E; 0], rows: pivot rows by pivot column, then the
 * non-selected rows ascending. */
gfech_status gfech_expand_rref(const gfech_result* res, uint8_t* E, int64_t lde);
gfech_status gfech_expand_transform(const gfech_result* res, uint8_t* T, int64_t ldt);
/* Same into device buffers (work ordered on `stream`, complete on return). */
gfech_status gfech_expand_rref_dev(const gfech_result* res, uint8_t* E_dev, int64_t lde, void* stream);
gfech_status gfech_expand_transform_dev(const gfech_result* res, uint8_t* T_dev, int64_t ldt, void* stream);

/* Device pointers to the result's matrices (valid until gfech_result_free). */
typedef struct gfech_view {
    const uint8_t* R; int64_t ldr;     /* r x (n - r) */
    const uint8_t* M; int64_t ldm;     /* r x r */
    const uint8_t* K; int64_t ldk;     /* (m - r) x r */
    const int32_t* gamma;              /* r   */
    const int32_t* gamma_bar;          /* n - r */
    const int32_t* rho;                /* r   */
    const int32_t* rho_bar;            /* m - r */
} gfech_view;
gfech_status gfech_device_view(const gfech_result* res, gfech_view* view);

/* Work counters of the run (cost model of Section 5: a product (x by y)(y by z)
 * counts xyz multiply-adds, echelonising x by y of rank r counts xyr). */
typedef struct gfech_stats {
    double mac_cleardown;   /* ClearDown's MADs */
    double mac_ech;         /* ECH jobs */
    double mac_updaterow;   /* UpdateRow on the data blocks */
    double mac_trafo;       /* UpdateRowTrafo on the transformation blocks */
    double mac_clearup;     /* ClearUp (Step 3) */
    double gather_bytes;    /* bytes read + written by extracts, riffles and copies */
    int64_t layers, echs, gemms, launches, syncs;
    int64_t block_rows, block_cols;   /* a and b */
    /* with opts.profile: summed device time and launch count of the MAD
     * kernel, the ECH kernel and the extract / riffle / list kernels */
    double ms_mad, ms_ech, ms_small;
    int64_t launches_mad, launches_ech, launches_small;
    /* operand bytes of every MAD launched (A, B and C read once, D written
     * once), summed over the launches of the engine run that produced this
     * result */
    double mad_bytes;
    /* with opts.profile: multiply-adds of the MAD launches that were timed
     * (all of them at level 2, about a quarter at level 3) */
    double mac_mad_timed;
    int64_t variant;        /* the GFECH_WANT_* the result was computed for */
    /* ClearDowns whose ECH of the leading columns of a wide block left rows
     * unselected: tail_checks of them found those rows reduced to zero on the
     * remaining columns (the result stands, no second ECH); ech_reruns ran
     * the ECH again on the whole block (Section 2.3.2 splits ech by columns
     * the same way) */
    int64_t tail_checks, ech_reruns;
} gfech_stats;
gfech_status gfech_get_stats(const gfech_result* res, gfech_stats* stats);

void gfech_result_free(gfech_result* res);

/* ---------------------------------------------------------------- single jobs
 * The paper's jobs (Section 4.1) on caller-owned device buffers, for callers
 * that build their own task graphs and for per-kernel checks.  Inputs must
 * hold canonical residues < p (not checked: results are unspecified
 * otherwise); shapes, pointers and p are checked.  Work is ordered on
 * `stream` (a hipStream_t, NULL = default) and complete on return. */

/* MAD: D = (C + A * B) mod p.  A: M x K (lda); B: K x N (ldb), row t of B is
 * row brow[t] of the B buffer when brow != NULL (a device int32 array); C:
 * M x N (ldc) or NULL for zero, row x of C is row crow[x] when crow != NULL;
 * D: M x N (ldd).  D may equal C when crow == NULL and ldc == ldd; D must not
 * overlap A or B.  K <= 65536. */
gfech_status gfech_mad_dev(int64_t M, int64_t N, int64_t K, uint32_t p,
                           const uint8_t* A, int64_t lda,
                           const uint8_t* B, int64_t ldb, const int32_t* brow,
                           const uint8_t* C, int64_t ldc, const int32_t* crow,
                           uint8_t* D, int64_t ldd, void* stream);

/* Several independent MADs in one launch (same rules per entry). */
typedef struct gfech_mad_desc {
    int64_t M, N, K;
    uint32_t p, reserved;
    const uint8_t* A; int64_t lda;
    const uint8_t* B; int64_t ldb; const int32_t* brow;
    const uint8_t* C; int64_t ldc; const int32_t* crow;
    uint8_t* D; int64_t ldd;
} gfech_mad_desc;
gfech_status gfech_mad_batch_dev(int64_t count, const gfech_mad_desc* descs, void* stream);

/* gfech_mad_batch_dev, and *kernel_ms (host memory) receives the summed
 * execution time of its MAD kernel launches, taken from each dispatch's own
 * begin and end timestamps (the upload of the descriptor array and launch
 * gaps excluded).  Returns once the launches have finished.  For measuring
 * the product kernel in isolation. */
gfech_status gfech_mad_batch_dev_timed(int64_t count, const gfech_mad_desc* descs, void* stream,
                                       double* kernel_ms);

/* MAD over GF(2) on bit-packed rows (bit b of word w of a row = column
 * 64 w + b): D = (C + A * B) over GF(2), i.e. row i of D is row i of C XOR
 * the rows of B that row i of A selects.  A: M x K (lda words per row, its
 * bits past column K - 1 ignored); B: K x N (ldb words); C: M x N (ldc
 * words) or NULL for zero; D: M x N (ldd words).  Bits of B and C past column
 * N - 1 must be zero (those of D then are).  D may equal C (same ld); D must
 * not overlap A or B.  Computed by the method of the four Russians: tables of
 * the XOR combinations of 8 rows of B in LDS, selected by the bytes of A. */
gfech_status gfech_mad_gf2_dev(int64_t M, int64_t N, int64_t K, const uint64_t* A, int64_t lda, const uint64_t* B,
                               int64_t ldb, const uint64_t* C, int64_t ldc, uint64_t* D, int64_t ldd, void* stream);

/* ECH (Remark 2.3) of one block H (rows x cols, ldh) in device memory.  With
 * r = rank(H) (returned in *rank, host memory) the device outputs are
 *   prow[r]        row of the t-th pivot, pivots by increasing column
 *   qrow[rows - r] non-pivot rows ascending;  pcol[r] pivot columns ascending;
 *   qcol[cols - r] non-pivot columns ascending
 *   M (r x r, ldm), K ((rows - r) x r, ldk), R (r x (cols - r), ldr) with
 *   [[M,0],[K,1]] [H[prow]; H[qrow]] [H[:, pcol] | H[:, qcol]] = [[-1, R],[0,0]]
 * (columns of M and K follow prow).  Buffers must be sized for r = min(rows, cols).
 * rows + cols <= 8192. */
gfech_status gfech_ech_dev(const uint8_t* H, int64_t rows, int64_t cols, int64_t ldh, uint32_t p,
                           int32_t* prow, int32_t* qrow, int32_t* pcol, int32_t* qcol,
                           uint8_t* M, int64_t ldm, uint8_t* K, int64_t ldk, uint8_t* R, int64_t ldr,
                           int64_t* rank, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): gfech_ech_dev with
 * its workspace in a fixed device array of the library's instead of an
 * allocation.  The array holds GFECH_NOALLOC_SCRATCH_BYTES (16 MiB) on the
 * device the library was initialised on, allocated when the library's device
 * code is loaded and held until the process ends.  A block needs
 * rows * (cols + min(rows, cols)) bytes of it; a larger one gives
 * GFECH_E_TOO_BIG before any work is queued.  The call allocates nothing and
 * does not wait: its work is ordered on `stream`, and the rank is written to
 * device memory, *rank_dev (one int32), instead of being returned.  Every
 * call shares the one array and it keeps the last call's contents (the ECH
 * initialises what it reads): calls whose work overlaps on the device (on
 * different streams, or captured work replayed concurrently) race and give
 * wrong results.  The library initialises itself on its first call, which
 * allocates (its streams and descriptor ring): make any other call first,
 * e.g. gfech_backend_name(). */
#define GFECH_NOALLOC_SCRATCH_BYTES ((int64_t)16 << 20)
gfech_status gfech_ech_dev_noalloc(const uint8_t* H, int64_t rows, int64_t cols, int64_t ldh, uint32_t p,
                                   int32_t* prow, int32_t* qrow, int32_t* pcol, int32_t* qcol,
                                   uint8_t* M, int64_t ldm, uint8_t* K, int64_t ldk, uint8_t* R, int64_t ldr,
                                   int32_t* rank_dev, void* stream);

/* ---------------------------------------------------------------- serving
 * A server echelonises requests as they arrive (continuous batching).
 * Requests are sorted into size classes; per class a worker thread keeps
 * every admitted request's block state in device memory and advances all of
 * them together, one phase of the method each per iteration, so requests
 * submitted while others run join at the next iteration and their jobs share
 * launches, while the classes run side by side on streams of their own.
 * Requests are admitted in arrival order within their class while the device
 * memory they hold (an upper bound per request) fits the budget, which the
 * classes share; a request whose bound alone exceeds the budget is refused.
 * Results are the same as from gfech_echelonise_u8 on the same input (the
 * default blocking).  The functions are thread-safe. */
typedef struct gfech_server gfech_server;
typedef struct gfech_server_cfg {
    int64_t hbm_budget_bytes;   /* device memory for admitted requests; 0 = 200 GB */
    int32_t max_active;         /* requests in flight at once; 0 = no limit but the budget */
    int32_t size_classes;       /* 1, 2 or 3 (0 = 3): requests are sorted by max(m, n) into
                                   classes (up to 512, up to 2048, larger; with 2 classes up to
                                   512 and larger), each with its own engine, streams and worker
                                   thread, so small requests never wait for the phases of large
                                   ones; admission is first come first served within a class
                                   against the one budget */
    int32_t reserved[4];
} gfech_server_cfg;
gfech_status gfech_server_create(const gfech_server_cfg* cfg, gfech_server** out);
/* Queue one problem.  The input (host or device memory, as the flag says) is
 * checked (entries < p) and copied before the call returns (a device input on
 * a stream of the server's own, waited for), so the caller may reuse its
 * buffer at once; *ticket names the request.  GFECH_E_TOO_BIG: the request
 * alone exceeds the budget (refused before anything is copied). */
gfech_status gfech_server_submit(gfech_server* srv, const gfech_problem* prob, int32_t input_on_device,
                                 uint64_t* ticket);
/* Non-blocking: *out receives the result of a finished request (the caller
 * owns it) or NULL while it is queued or running.  A ticket is answered once;
 * unknown tickets give GFECH_E_ARG, failed requests their error status. */
gfech_status gfech_server_poll(gfech_server* srv, uint64_t ticket, gfech_result** out);
/* Cancels a request: a queued one is dropped at once, a running one stops at
 * its next phase boundary (its device work completes, its memory is freed).
 * Its ticket then answers GFECH_E_CANCELLED (unless it had already finished,
 * in which case its result stays available).  Unknown tickets: GFECH_E_ARG. */
gfech_status gfech_server_cancel(gfech_server* srv, uint64_t ticket);
/* Blocking form of gfech_server_poll. */
gfech_status gfech_server_wait(gfech_server* srv, uint64_t ticket, gfech_result** out);
/* Counters of a server since its creation: the largest device-memory
 * footprint of the requests in flight at once (the bounds admission uses,
 * never above the budget), the most requests in flight at once, and the
 * requests admitted and finished. */
typedef struct gfech_server_stats {
    int64_t peak_bytes_in_flight;
    int64_t peak_active;
    int64_t admitted, finished;
} gfech_server_stats;
gfech_status gfech_server_get_stats(gfech_server* srv, gfech_server_stats* stats);
/* Drops queued requests, lets running ones finish, frees unclaimed results. */
void gfech_server_destroy(gfech_server* srv);

const char* gfech_strerror(gfech_status s);
/* Detail of the last failure on this thread ("" if none). */
const char* gfech_last_error(void);
/* Name of the compute backend this library was built with ("hip-gfx950"). */
const char* gfech_backend_name(void);

#ifdef __cplusplus
}
#endif
#endif /* GFECH_H */
