// HIP backend for gfx950 (MI355X): the kernels behind the planner's grouped
// jobs, and the device-memory / stream plumbing.
//
//  - k_gemm_modp   MAD / MUL mod p (the O(n^3) work of UpdateRow,
//                  UpdateRowTrafo, ClearDown and ClearUp) on int8 MFMA
//                  (v_mfma_i32_16x16x64_i8) with int32 accumulation; one
//                  launch runs every descriptor of a phase.
//  - k_ech         ECH (Remark 2.3): one workgroup per block.
//  - k_gather, k_fill, k_lists, k_sort, k_range: extracts, riffles and the
//                  index-list jobs (HBM-bound).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "backend.h"

namespace gfech {
namespace {

// ============================================================================ field helpers

// x mod p for 0 <= x < 2^24, p <= 251: q = floor(x * floor(2^24 / p) / 2^24) is
// floor(x / p) or one less, so one conditional subtraction finishes.
__device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t p, uint32_t minv) {
    uint32_t q = __umulhi(x << 8, minv);
    uint32_t r = x - q * p;
    return r >= p ? r - p : r;
}

// v mod p for any int32 v with |v| < 2^31 - 256: shift by a multiple of p into
// [0, 2^32), then q = mulhi(u, floor(2^32 / p)) is floor(u / p) or one less.
struct ModP {
    uint32_t p, m, bias;
    __device__ __forceinline__ explicit ModP(uint32_t pp)
        : p(pp), m((uint32_t)(0x100000000ull / pp)), bias((uint32_t)((0x80000000u / pp) * pp)) {}
    __device__ __forceinline__ uint32_t operator()(int v) const {
        uint32_t u = (uint32_t)v + bias;
        uint32_t r = u - __umulhi(u, m) * p;
        return r >= p ? r - p : r;
    }
};

// ============================================================================ GEMM mod p

constexpr int TM = 128;          // rows of D per workgroup tile
constexpr int TN = 128;          // columns of D per workgroup tile
constexpr int TK = 64;           // reduction depth per LDS stage
constexpr int LDS_ROW = 80;      // bytes per LDS row (64 data + 16 pad)
constexpr int GEMM_THREADS = 256;

typedef int v4i __attribute__((ext_vector_type(4)));

struct GemmTileMap {           // per-descriptor tile grid, device side
    int32_t tiles_n;           // tiles along N
    int32_t first_tile;        // prefix sum of tiles
};

// 16 bytes starting at any byte address p, of which `rem` (>= 1) are valid.
// Rows with at least 20 valid bytes left are read as aligned dwords and
// realigned (every byte read lies inside the row); shorter tails are read byte
// by byte, so nothing past the last valid byte is ever touched.
__device__ __forceinline__ uint4 load16_lim(const uint8_t* p, int rem) {
    if (rem >= 20) {
        uintptr_t a = (uintptr_t)p;
        const uint32_t* q = (const uint32_t*)(a & ~(uintptr_t)3);
        uint32_t sh = (uint32_t)(a & 3);
        uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
        if (sh == 0) return make_uint4(w0, w1, w2, w3);
        uint32_t w4 = q[4];
        return make_uint4(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
                          __builtin_amdgcn_alignbyte(w3, w2, sh), __builtin_amdgcn_alignbyte(w4, w3, sh));
    }
    uint32_t w[4] = {0, 0, 0, 0};
    int n = rem < 16 ? rem : 16;
    for (int b = 0; b < n; ++b) w[b >> 2] |= (uint32_t)p[b] << (8 * (b & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// 8 bytes starting at p, `rem` (>= 1) valid; same rules as load16_lim
__device__ __forceinline__ uint2 load8_lim(const uint8_t* p, int rem) {
    if (rem >= 12) {
        uintptr_t a = (uintptr_t)p;
        const uint32_t* q = (const uint32_t*)(a & ~(uintptr_t)3);
        uint32_t sh = (uint32_t)(a & 3);
        uint32_t w0 = q[0], w1 = q[1];
        if (sh == 0) return make_uint2(w0, w1);
        uint32_t w2 = q[2];
        return make_uint2(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh));
    }
    uint32_t w[2] = {0, 0};
    int n = rem < 8 ? rem : 8;
    for (int b = 0; b < n; ++b) w[b >> 2] |= (uint32_t)p[b] << (8 * (b & 3));
    return make_uint2(w[0], w[1]);
}

// residues of p > 127 become signed int8 values x - p for x >= 128: add 256 - p to those bytes
__device__ __forceinline__ uint32_t centre(uint32_t w, uint32_t adj) {
    uint32_t hi = (w >> 7) & 0x01010101u;
    return w + hi * adj;
}

__global__ void __launch_bounds__(GEMM_THREADS)
k_gemm_modp(const GemmDesc* __restrict__ descs, const GemmTileMap* __restrict__ maps, int ndesc) {
    __shared__ __attribute__((aligned(16))) uint8_t As[TM * LDS_ROW];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * LDS_ROW];   // transposed: [n][k]

    // which descriptor owns this tile (binary search over the prefix sums)
    const int tile = blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (maps[mid].first_tile <= tile) lo = mid; else hi = mid - 1;
    }
    const GemmDesc g = descs[lo];
    const int local = tile - maps[lo].first_tile;
    const int tn = maps[lo].tiles_n;
    const int m0 = (local / tn) * TM;
    const int n0 = (local % tn) * TN;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * 64;      // wave's 64 x 64 sub-tile
    const int wn = (wave & 1) * 64;
    const uint32_t p = (uint32_t)g.p;
    const uint32_t adj = p > 127 ? 256u - p : 0u;

    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};

    for (int k0 = 0; k0 < g.K; k0 += TK) {
        // ---- A tile: 128 rows x 64 bytes, two 16-byte chunks per thread
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int c = tid + s * GEMM_THREADS;
            int row = c >> 2;
            int kc = (c & 3) * 16;
            uint4 v = make_uint4(0, 0, 0, 0);
            int gr = m0 + row, gk = k0 + kc;
            if (gr < g.M && gk < g.K) {
                v = load16_lim(g.A + (int64_t)gr * g.lda + gk, g.K - gk);
                if (adj) { v.x = centre(v.x, adj); v.y = centre(v.y, adj); v.z = centre(v.z, adj); v.w = centre(v.w, adj); }
            }
            *(uint4*)(As + row * LDS_ROW + kc) = v;
        }
        // ---- B tile: 64 k-rows x 128 columns, stored transposed; each thread 4 k x 8 n
        {
            int kg = tid >> 4;           // 0..15 -> k rows 4kg..4kg+3
            int ng = tid & 15;           // 0..15 -> columns 8ng..8ng+7
            uint32_t lo4[4], hi4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int gk = k0 + kg * 4 + t;
                int gn = n0 + ng * 8;
                uint2 v = make_uint2(0, 0);
                if (gk < g.K && gn < g.N) {
                    int64_t br = g.brow ? g.brow[gk] : gk;
                    v = load8_lim(g.B + br * g.ldb + gn, g.N - gn);
                    if (adj) { v.x = centre(v.x, adj); v.y = centre(v.y, adj); }
                }
                lo4[t] = v.x;
                hi4[t] = v.y;
            }
            // transpose 4 (k) x 8 (n) bytes: column j gathers byte j of each k-row
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint32_t sh = (j & 3) * 8;
                const uint32_t* src = j < 4 ? lo4 : hi4;
                uint32_t col = ((src[0] >> sh) & 0xffu) | (((src[1] >> sh) & 0xffu) << 8) |
                               (((src[2] >> sh) & 0xffu) << 16) | (((src[3] >> sh) & 0xffu) << 24);
                *(uint32_t*)(Bs + (ng * 8 + j) * LDS_ROW + kg * 4) = col;
            }
        }
        __syncthreads();
        // ---- MFMA: each wave 4 x 4 blocks of 16 x 16, k = 64
        const int r16 = lane & 15;
        const int kq = (lane >> 4) * 16;
        v4i af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = *(const v4i*)(As + (wm + i * 16 + r16) * LDS_ROW + kq);
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = *(const v4i*)(Bs + (wn + j * 16 + r16) * LDS_ROW + kq);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bf[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

    // ---- epilogue: D = (Cin + acc) mod p
    // acc[i][j] element e sits at row 4 * (lane / 16) + e, column lane % 16 of block (i, j);
    // |acc| <= K * 127^2 < 2^30 for K <= 2^16
    const ModP mod(p);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int row = m0 + wm + i * 16 + (lane >> 4) * 4 + e;
                int col = n0 + wn + j * 16 + (lane & 15);
                if (row < g.M && col < g.N) {
                    int v = acc[i][j][e];
                    if (g.C) {
                        int64_t cr = g.crow ? g.crow[row] : row;
                        v += g.C[cr * g.ldc + col];
                    }
                    g.D[(int64_t)row * g.ldd + col] = (uint8_t)mod(v);
                }
            }
}

// ============================================================================ ECH

constexpr int ECH_THREADS = 256;

__device__ __forceinline__ uint32_t pow_mod_dev(uint32_t a, uint32_t e, uint32_t p) {
    uint32_t r = 1, b = a % p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return r;
}

// dynamic LDS: sel[rows] flags, f[rows] multipliers, prow_lds[cols + maxr] pivot row copy
__global__ void __launch_bounds__(ECH_THREADS) k_ech(const EchDesc* __restrict__ descs) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    __shared__ int red[ECH_THREADS / 64];
    __shared__ uint32_t s_scale;
    const EchDesc e = descs[blockIdx.x];
    const int rows = e.rows, cols = e.cols;
    const int maxr = rows < cols ? rows : cols;
    const int width = cols + maxr;
    const uint32_t p = (uint32_t)e.p;
    const uint32_t minv = (1u << 24) / p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint8_t* sel = smem;                        // rows
    uint8_t* f = smem + rows;                   // rows
    uint8_t* prow_l = smem + 2 * rows;          // width
    int* piv_rows = (int*)(smem + ((2 * rows + width + 15) & ~15));   // maxr
    int* piv_cols = piv_rows + maxr;

    for (int x = tid; x < rows; x += ECH_THREADS) sel[x] = 0;
    for (int64_t idx = tid; idx < (int64_t)rows * width; idx += ECH_THREADS) {
        int x = (int)(idx / width), y = (int)(idx % width);
        e.work[(int64_t)x * e.ldw + y] = y < cols ? e.H[(int64_t)x * e.ldh + y] : 0;
    }
    __syncthreads();

    int r = 0;
    for (int c = 0; c < cols && r < maxr; ++c) {
        // first not-yet-selected row with a non-zero in column c
        int best = 0x7fffffff;
        for (int x = tid; x < rows; x += ECH_THREADS)
            if (!sel[x] && e.work[(int64_t)x * e.ldw + c]) { best = x; break; }
        for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
        if (lane == 0) red[wave] = best;
        __syncthreads();
        best = red[0];
        for (int w = 1; w < ECH_THREADS / 64; ++w) best = min(best, red[w]);
        if (best == 0x7fffffff) {
            __syncthreads();
            continue;
        }
        const int piv = best;
        uint8_t* P = e.work + (int64_t)piv * e.ldw;
        if (tid == 0) {
            uint32_t v = P[c];
            s_scale = (p - pow_mod_dev(v, p - 2, p)) % p;   // pivot becomes -1
            P[cols + r] = 1;                                 // its own transformation column
            sel[piv] = 1;
            piv_rows[r] = piv;
            piv_cols[r] = c;
        }
        __syncthreads();
        const uint32_t s = s_scale;
        for (int y = c + tid; y < cols + r + 1; y += ECH_THREADS) {   // data columns c.. and T columns 0..r
            uint32_t v = mod_small(P[y] * s, p, minv);
            P[y] = (uint8_t)v;
            prow_l[y] = (uint8_t)v;
        }
        for (int x = tid; x < rows; x += ECH_THREADS) f[x] = x == piv ? 0 : e.work[(int64_t)x * e.ldw + c];
        __syncthreads();
        // row x += f[x] * pivot row, on columns c..cols-1 and transformation columns 0..r
        const int span = cols - c;
        const int wtot = span + r + 1;
        for (int x = wave; x < rows; x += ECH_THREADS / 64) {
            uint32_t fx = f[x];
            if (!fx) continue;
            uint8_t* W = e.work + (int64_t)x * e.ldw;
            for (int t = lane; t < wtot; t += 64) {
                int y = t < span ? c + t : cols + (t - span);
                W[y] = (uint8_t)mod_small(W[y] + fx * prow_l[y], p, minv);
            }
        }
        __syncthreads();
        ++r;
    }
    __syncthreads();
    // ---- outputs
    if (tid == 0) *e.rcount = r;
    for (int t = tid; t < r; t += ECH_THREADS) {
        e.prow[t] = piv_rows[t];
        e.pcol[t] = piv_cols[t];
    }
    // reuse f[] as "column is a pivot" flags (cols <= rows is not guaranteed: use prow_l)
    for (int y = tid; y < cols; y += ECH_THREADS) prow_l[y] = 0;
    __syncthreads();
    for (int t = tid; t < r; t += ECH_THREADS) prow_l[piv_cols[t]] = 1;
    __syncthreads();
    if (tid == 0) {
        int q = 0;
        for (int x = 0; x < rows; ++x)
            if (!sel[x]) e.qrow[q++] = x;
        q = 0;
        for (int y = 0; y < cols; ++y)
            if (!prow_l[y]) e.qcol[q++] = y;
    }
    __syncthreads();
    // Mo[t][u] = T[prow[t]][u];  Ro[t][k] = W[prow[t]][qcol[k]];  Ko[s][u] = T[qrow[s]][u]
    for (int64_t idx = tid; idx < (int64_t)r * r; idx += ECH_THREADS) {
        int t = (int)(idx / r), u = (int)(idx % r);
        e.Mo[(int64_t)t * e.ldm + u] = e.work[(int64_t)piv_rows[t] * e.ldw + cols + u];
    }
    const int nr = cols - r;
    for (int64_t idx = tid; idx < (int64_t)r * nr; idx += ECH_THREADS) {
        int t = (int)(idx / nr), k = (int)(idx % nr);
        e.Ro[(int64_t)t * e.ldr + k] = e.work[(int64_t)piv_rows[t] * e.ldw + e.qcol[k]];
    }
    const int nq = rows - r;
    for (int64_t idx = tid; idx < (int64_t)nq * r; idx += ECH_THREADS) {
        int s2 = (int)(idx / r), u = (int)(idx % r);
        e.Ko[(int64_t)s2 * e.ldk + u] = e.work[(int64_t)e.qrow[s2] * e.ldw + cols + u];
    }
}

// ---------------------------------------------------------------------------- ECH, panel form
//
// One workgroup per block, one thread per row (rows <= 512).  Columns are
// processed in panels of PW: the thread holds its row's panel entries and its
// row of the panel transform F in registers as unreduced 32-bit sums (each
// elimination is one multiply-add; values stay below 2^24 for PW <= 32 and
// p <= 251).  A pivot is the first not-yet-selected row with a non-zero in
// the column (the paper's rule); each wave proposes its first candidate and
// parks that row in LDS, and the winning row is reduced by its wave and read
// by all.  After a panel, every other column of the block and every
// transformation column of earlier pivots gets
//     W[x] := (x a pivot of this panel ? 0 : W[x]) + F[x] * W_old[pivot rows]
// on int8 MFMA; the transformation columns of the new pivots are F itself.
constexpr int PW = 32;          // panel width
constexpr int FL_ROW = 80;      // LDS bytes per row of F (64 used by the MFMA, zero beyond the panel)
constexpr int VCH = 64;         // columns per trailing-update chunk
constexpr int ECHP_MAX_ROWS = 512;

__host__ __device__ constexpr size_t echp_fixed_lds() {
    return 128 + 2 * 16 * 64 * 4 + 2 * ECHP_MAX_ROWS * 4 + 256 * 4 + 2 * ECHP_MAX_ROWS + VCH * FL_ROW;
}
__host__ __device__ inline size_t echp_lds_bytes(int rows) { return echp_fixed_lds() + (size_t)((rows + 15) & ~15) * FL_ROW; }

__global__ void __launch_bounds__(512) k_ech_panel(const EchDesc* __restrict__ descs) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const EchDesc e = descs[blockIdx.x];
    const int rows = e.rows, cols = e.cols;
    const int maxr = rows < cols ? rows : cols;
    const int width = cols + maxr;
    const uint32_t p = (uint32_t)e.p;
    const uint32_t minv = (1u << 24) / p;
    const uint32_t adj = p > 127 ? 256u - p : 0u;
    const ModP mod(p);
    const int x = threadIdx.x;
    const int nthr = blockDim.x, lane = x & 63, wave = x >> 6, nwaves = nthr >> 6;
    const int rows16 = (rows + 15) & ~15;

    int* cand = (int*)smem;                                        // [2][16]
    uint32_t* slot = (uint32_t*)(smem + 128);                      // [2][16][64]
    int* prl = (int*)(smem + 128 + 2 * 16 * 64 * 4);               // pivot rows, pivot order
    int* pcl = prl + ECHP_MAX_ROWS;                                // pivot columns
    uint32_t* invt = (uint32_t*)(pcl + ECHP_MAX_ROWS);             // inverses mod p
    uint8_t* sel = (uint8_t*)(invt + 256);                         // row selected
    uint8_t* inpanel = sel + ECHP_MAX_ROWS;                        // row selected in the current panel
    uint8_t* Vt = inpanel + ECHP_MAX_ROWS;                         // [VCH][FL_ROW] pivot rows, transposed
    uint8_t* Fl = Vt + VCH * FL_ROW;                               // [rows16][FL_ROW]

    for (int i = x; i < 256; i += nthr) invt[i] = (i > 0 && (uint32_t)i < p) ? pow_mod_dev((uint32_t)i, p - 2, p) : 0u;
    for (int i = x; i < ECHP_MAX_ROWS; i += nthr) sel[i] = 0;
    for (int64_t idx = x; idx < (int64_t)rows * width; idx += nthr) {
        int rr = (int)(idx / width), y = (int)(idx % width);
        e.work[(int64_t)rr * e.ldw + y] = y < cols ? e.H[(int64_t)rr * e.ldh + y] : 0;
    }
    __syncthreads();
    uint8_t* Wx = e.work + (int64_t)x * e.ldw;

    int r = 0;
    for (int c0 = 0; c0 < cols && r < maxr; c0 += PW) {
        const int wc = min(PW, cols - c0);
        uint32_t reg[PW], F[PW];
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            reg[j] = (x < rows && j < wc) ? Wx[c0 + j] : 0u;
            F[j] = 0;
        }
        bool mysel = x < rows && sel[x];
        bool mine = false;
        uint32_t myscale = 0;
        int rp = 0;
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            if (k < wc && r + rp < maxr) {
                const uint32_t v = mod_small(reg[k], p, minv);
                reg[k] = v;
                const bool isc = x < rows && !mysel && v != 0;
                const unsigned long long bal = __ballot(isc);
                const int par = k & 1;
                if (bal) {
                    const int first = __ffsll((long long)bal) - 1;
                    if (lane == first) {
                        cand[par * 16 + wave] = x;
                        uint32_t* my = slot + (par * 16 + wave) * 64;
#pragma unroll
                        for (int j = 0; j < PW; ++j) my[j] = reg[j];
#pragma unroll
                        for (int t = 0; t < PW; ++t) my[PW + t] = (t == rp) ? 1u : F[t];
                    }
                } else if (lane == 0) {
                    cand[par * 16 + wave] = 0x7fffffff;
                }
                __syncthreads();
                int best = 0x7fffffff;
                for (int w = 0; w < nwaves; ++w) best = min(best, cand[par * 16 + w]);
                if (best != 0x7fffffff) {
                    uint32_t* ps = slot + (par * 16 + (best >> 6)) * 64;
                    if (wave == (best >> 6)) ps[lane] = mod_small(ps[lane], p, minv);
                    __syncthreads();
                    const uint32_t s = (p - invt[ps[k]]) % p;        // -1 / pivot
                    if (x == best) {
                        mysel = true;
                        mine = true;
                        myscale = s;
#pragma unroll
                        for (int t = 0; t < PW; ++t)
                            if (t == rp) F[t] = 1;
                        sel[x] = 1;
                        prl[r + rp] = x;
                        pcl[r + rp] = c0 + k;
                    } else if (x < rows) {
                        const uint32_t f = mod_small(v * s, p, minv);
                        if (f) {
#pragma unroll
                            for (int j = k + 1; j < PW; ++j) reg[j] += f * ps[j];
                            reg[k] = 0;
#pragma unroll
                            for (int t = 0; t < PW; ++t) F[t] += f * ps[PW + t];
                        }
                    }
                    ++rp;
                }
            }
        }
        // normalise this panel's pivot rows (pivot -> -1) and reduce everything
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            uint32_t a = mod_small(reg[j], p, minv), b = mod_small(F[j], p, minv);
            if (mine) {
                a = mod_small(a * myscale, p, minv);
                b = mod_small(b * myscale, p, minv);
            }
            reg[j] = a;
            F[j] = b;
        }
        if (x < rows) {
#pragma unroll
            for (int j = 0; j < PW; ++j)
                if (j < wc) Wx[c0 + j] = (uint8_t)reg[j];
#pragma unroll
            for (int t = 0; t < PW; ++t)
                if (t < rp) Wx[cols + r + t] = (uint8_t)F[t];
            inpanel[x] = mine ? 1 : 0;
        }
        if (x < rows16) {
            uint32_t* fr = (uint32_t*)(Fl + x * FL_ROW);
#pragma unroll
            for (int w4 = 0; w4 < 16; ++w4) {
                uint32_t word = 0;
                if (x < rows) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int t = w4 * 4 + b;
                        if (t < PW && t < rp) word |= F[t < PW ? t : 0] << (8 * b);
                    }
                }
                fr[w4] = adj ? centre(word, adj) : word;
            }
        }
        __syncthreads();
        if (rp > 0) {
            const int nd = cols - (c0 + wc);     // data columns right of the panel
            const int total = nd + r;            // plus transformation columns of earlier pivots
            for (int ch = 0; ch < total; ch += VCH) {
                for (int i = x; i < VCH * 16; i += nthr) {
                    const int cl = i >> 4, tw = (i & 15) * 4, q = ch + cl;
                    uint32_t word = 0;
                    if (q < total) {
                        const int y = q < nd ? c0 + wc + q : cols + (q - nd);
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int t = tw + b;
                            if (t < rp) word |= (uint32_t)e.work[(int64_t)prl[r + t] * e.ldw + y] << (8 * b);
                        }
                    }
                    *(uint32_t*)(Vt + cl * FL_ROW + tw) = adj ? centre(word, adj) : word;
                }
                __syncthreads();
                const int nb = (rows16 >> 4) * (VCH / 16);
                for (int b = wave; b < nb; b += nwaves) {
                    const int rb = b / (VCH / 16), cb = b % (VCH / 16);
                    const v4i av = *(const v4i*)(Fl + (rb * 16 + (lane & 15)) * FL_ROW + (lane >> 4) * 16);
                    const v4i bv = *(const v4i*)(Vt + (cb * 16 + (lane & 15)) * FL_ROW + (lane >> 4) * 16);
                    const v4i acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, v4i{0, 0, 0, 0}, 0, 0, 0);
                    const int cl = cb * 16 + (lane & 15), q = ch + cl;
                    if (q < total) {
                        const int y = q < nd ? c0 + wc + q : cols + (q - nd);
#pragma unroll
                        for (int ee = 0; ee < 4; ++ee) {
                            const int row = rb * 16 + (lane >> 4) * 4 + ee;
                            if (row < rows) {
                                uint8_t* w = e.work + (int64_t)row * e.ldw + y;
                                const int old = inpanel[row] ? 0 : (int)*w;
                                *w = (uint8_t)mod(acc[ee] + old);
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        r += rp;
    }
    __syncthreads();
    // ---- outputs
    if (x == 0) *e.rcount = r;
    for (int t = x; t < r; t += nthr) {
        e.prow[t] = prl[t];
        e.pcol[t] = pcl[t];
    }
    if (x == 0) {
        int q = 0;
        for (int rr = 0; rr < rows; ++rr)
            if (!sel[rr]) e.qrow[q++] = rr;
        q = 0;
        int t = 0;
        for (int y = 0; y < cols; ++y) {
            if (t < r && pcl[t] == y) { ++t; continue; }
            e.qcol[q++] = y;
        }
    }
    __syncthreads();
    for (int64_t idx = x; idx < (int64_t)r * r; idx += nthr) {
        int t = (int)(idx / r), u = (int)(idx % r);
        e.Mo[(int64_t)t * e.ldm + u] = e.work[(int64_t)prl[t] * e.ldw + cols + u];
    }
    const int nr = cols - r;
    for (int64_t idx = x; idx < (int64_t)r * nr; idx += nthr) {
        int t = (int)(idx / nr), k2 = (int)(idx % nr);
        e.Ro[(int64_t)t * e.ldr + k2] = e.work[(int64_t)prl[t] * e.ldw + e.qcol[k2]];
    }
    const int nq = rows - r;
    for (int64_t idx = x; idx < (int64_t)nq * r; idx += nthr) {
        int s2 = (int)(idx / r), u = (int)(idx % r);
        e.Ko[(int64_t)s2 * e.ldk + u] = e.work[(int64_t)e.qrow[s2] * e.ldw + cols + u];
    }
}

// ============================================================================ small jobs

constexpr int SMALL_THREADS = 256;

// grid: (x blocks striding over elements, y = descriptor)
__global__ void __launch_bounds__(SMALL_THREADS) k_gather(const GatherDesc* __restrict__ descs) {
    const GatherDesc g = descs[blockIdx.y];
    const int64_t total = (int64_t)g.rows * g.cols;
    if (total == 0) return;
    for (int64_t idx = (int64_t)blockIdx.x * SMALL_THREADS + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * SMALL_THREADS) {
        int x = (int)(idx / g.cols), y = (int)(idx % g.cols);
        int64_t sr = g.srow ? g.srow[x] : x, sc = g.scol ? g.scol[y] : y;
        uint32_t v = g.src[sr * g.lds + sc];
        if (g.neg_p) v = (uint32_t)((g.neg_p - (int)v) % g.neg_p);
        int64_t dr = g.drow ? g.drow[x] : x, dc = g.dcol ? g.dcol[y] : y;
        g.dst[dr * g.ldd + dc] = (uint8_t)v;
    }
}

__global__ void __launch_bounds__(SMALL_THREADS) k_fill(const FillDesc* __restrict__ descs) {
    const FillDesc f = descs[blockIdx.y];
    if (f.dcol) {
        for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < f.rows; t += gridDim.x * SMALL_THREADS)
            f.dst[(int64_t)t * f.ldd + f.dcol[t]] = (uint8_t)f.diag_value;
        return;
    }
    const int64_t total = (int64_t)f.rows * f.cols;
    for (int64_t idx = (int64_t)blockIdx.x * SMALL_THREADS + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * SMALL_THREADS) {
        int x = (int)(idx / f.cols), y = (int)(idx % f.cols);
        f.dst[(int64_t)x * f.ldd + y] = (uint8_t)((x == y && f.diag_value >= 0) ? f.diag_value : f.value);
    }
}

__global__ void __launch_bounds__(SMALL_THREADS) k_lists(const ListDesc* __restrict__ descs) {
    const ListDesc l = descs[blockIdx.y];
    for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < l.npick; t += gridDim.x * SMALL_THREADS)
        l.append[t] = l.add + l.map[l.pick ? l.pick[t] : t];
    for (int s = blockIdx.x * SMALL_THREADS + threadIdx.x; s < l.nkeep; s += gridDim.x * SMALL_THREADS)
        l.keep_out[s] = l.map[l.keep ? l.keep[s] : s];
}

// rank sort of distinct values: out[rank(t)] = add + (mode ? t : vals[t])
__global__ void __launch_bounds__(SMALL_THREADS) k_sort(const SortDesc* __restrict__ descs) {
    const SortDesc s = descs[blockIdx.y];
    for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < s.n; t += gridDim.x * SMALL_THREADS) {
        int v = s.vals[t], rank = 0;
        for (int u = 0; u < s.n; ++u) rank += s.vals[u] < v;
        s.out[rank] = s.add + (s.mode ? t : v);
    }
}

__global__ void __launch_bounds__(SMALL_THREADS)
k_range(const uint8_t* __restrict__ A, int64_t m, int64_t n, int64_t lda, int p, unsigned long long* bad) {
    unsigned long long cnt = 0;
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * SMALL_THREADS + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * SMALL_THREADS) {
        int64_t x = idx / n, y = idx % n;
        cnt += A[x * lda + y] >= p;
    }
    if (cnt) atomicAdd(bad, cnt);
}

// ============================================================================ host side

constexpr size_t kPad = 256;                 // tail padding of every allocation (vector over-read)
constexpr size_t kRing = 64ull << 20;        // descriptor staging ring

#define HIP_OK(expr)                                                            \
    do {                                                                        \
        hipError_t _e = (expr);                                                 \
        if (_e != hipSuccess) { note_error(_e, #expr); }                        \
    } while (0)

class HipBackend final : public Backend {
public:
    bool init(std::string* err) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
            if (err) *err = "no HIP device";
            return false;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
            if (err) *err = "hipGetDeviceProperties failed";
            return false;
        }
        if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) {
            if (err) *err = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
            return false;
        }
        num_cu_ = prop.multiProcessorCount;
        if (hipHostMalloc(&ring_host_, kRing) != hipSuccess || hipMalloc(&ring_dev_, kRing) != hipSuccess) {
            if (err) *err = "descriptor ring allocation failed";
            return false;
        }
        if (hipMalloc(&counter_, 64) != hipSuccess) {
            if (err) *err = "counter allocation failed";
            return false;
        }
        if (hipFuncSetAttribute((const void*)k_ech_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)echp_lds_bytes(ECHP_MAX_ROWS)) != hipSuccess) {
            if (err) *err = "cannot reserve LDS for the ECH kernel";
            return false;
        }
        return true;
    }

    const char* name() const override { return "hip-gfx950"; }

    void* alloc(size_t bytes) override {
        void* p = nullptr;
        size_t want = bytes + kPad;
        auto it = free_.lower_bound(want);
        if (it != free_.end() && it->first <= 2 * want + (64u << 20)) {
            p = it->second;
            sizes_[p] = it->first;
            free_.erase(it);
            return p;
        }
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            trim();
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        sizes_[p] = want;
        return p;
    }
    void release(void* p) override {
        if (!p) return;
        auto it = sizes_.find(p);
        if (it == sizes_.end()) return;
        free_.insert({it->second, p});
        sizes_.erase(it);
    }
    void trim() {
        hipStreamSynchronize(stream_);
        for (auto& kv : free_) hipFree(kv.second);
        free_.clear();
    }
    void zero(void* p, size_t bytes) override {
        if (bytes) HIP_OK(hipMemsetAsync(p, 0, bytes, stream_));
    }
    void upload(void* dst, const void* src, size_t bytes) override {
        if (!bytes) return;
        if (bytes <= kRing / 4) {
            void* h = stage(src, bytes);
            HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream_));
        } else {
            HIP_OK(hipStreamSynchronize(stream_));
            HIP_OK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        }
    }
    void download(void* dst, const void* src, size_t bytes) override {
        if (!bytes) return;
        HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream_));
        HIP_OK(hipStreamSynchronize(stream_));
    }
    void copy(void* dst, const void* src, size_t bytes) override {
        if (bytes) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream_));
    }
    void sync() override { HIP_OK(hipStreamSynchronize(stream_)); }
    void set_stream(void* s) override { stream_ = (hipStream_t)s; }
    int error() const override { return err_; }

    void gemm(const std::vector<GemmDesc>& ds) override {
        std::vector<GemmDesc> d;
        std::vector<GemmTileMap> maps;
        int64_t tiles = 0;
        for (const GemmDesc& g : ds) {
            if (g.M <= 0 || g.N <= 0) continue;
            if (g.K > 65536) { note_error(hipErrorInvalidValue, "gemm K > 65536"); return; }
            GemmTileMap t;
            t.tiles_n = (g.N + TN - 1) / TN;
            t.first_tile = (int32_t)tiles;
            tiles += (int64_t)((g.M + TM - 1) / TM) * t.tiles_n;
            d.push_back(g);
            maps.push_back(t);
        }
        if (d.empty()) return;
        if (tiles > INT32_MAX) { note_error(hipErrorInvalidValue, "too many gemm tiles"); return; }
        const GemmDesc* dd = (const GemmDesc*)put(d.data(), d.size() * sizeof(GemmDesc));
        const GemmTileMap* dm = (const GemmTileMap*)put(maps.data(), maps.size() * sizeof(GemmTileMap));
        hipEvent_t e0 = prof_begin();
        hipLaunchKernelGGL(k_gemm_modp, dim3((unsigned)tiles), dim3(GEMM_THREADS), 0, stream_, dd, dm, (int)d.size());
        HIP_OK(hipGetLastError());
        prof_end(0, e0);
    }

    void ech(const std::vector<EchDesc>& ds) override {
        if (ds.empty()) return;
        int maxrows_all = 0;
        for (const EchDesc& e : ds) maxrows_all = std::max(maxrows_all, e.rows);
        if (maxrows_all <= ECHP_MAX_ROWS && !getenv("GFECH_ECH_SIMPLE")) {
            int threads = std::max(64, (maxrows_all + 63) / 64 * 64);
            size_t shm = echp_lds_bytes(maxrows_all);
            const EchDesc* dd = (const EchDesc*)put(ds.data(), ds.size() * sizeof(EchDesc));
            hipEvent_t e0 = prof_begin();
            hipLaunchKernelGGL(k_ech_panel, dim3((unsigned)ds.size()), dim3(threads), shm, stream_, dd);
            HIP_OK(hipGetLastError());
            prof_end(1, e0);
            return;
        }
        int maxrows = 0, maxw = 0;
        for (const EchDesc& e : ds) {
            int maxr = std::min(e.rows, e.cols);
            maxrows = std::max(maxrows, e.rows);
            maxw = std::max(maxw, e.cols + maxr);
        }
        int maxr_all = 0;
        for (const EchDesc& e : ds) maxr_all = std::max(maxr_all, std::min(e.rows, e.cols));
        size_t shm = ((size_t)(2 * maxrows + maxw + 15) & ~(size_t)15) + 2 * sizeof(int) * (size_t)maxr_all;
        if (shm > 64 * 1024) { note_error(hipErrorInvalidValue, "ech block too large for LDS"); return; }
        const EchDesc* dd = (const EchDesc*)put(ds.data(), ds.size() * sizeof(EchDesc));
        hipEvent_t e0 = prof_begin();
        hipLaunchKernelGGL(k_ech, dim3((unsigned)ds.size()), dim3(ECH_THREADS), shm, stream_, dd);
        HIP_OK(hipGetLastError());
        prof_end(1, e0);
    }

    template <typename D, typename F>
    void small(const std::vector<D>& ds, F kernel, int64_t (*work)(const D&)) {
        if (ds.empty()) return;
        int64_t mx = 1;
        for (const D& x : ds) mx = std::max(mx, work(x));
        int64_t bx = std::min<int64_t>((mx + SMALL_THREADS - 1) / SMALL_THREADS, 4096);
        for (size_t off = 0; off < ds.size(); off += 65535) {
            size_t cnt = std::min<size_t>(65535, ds.size() - off);
            const D* dd = (const D*)put(ds.data() + off, cnt * sizeof(D));
            hipEvent_t e0 = prof_begin();
            hipLaunchKernelGGL(kernel, dim3((unsigned)bx, (unsigned)cnt), dim3(SMALL_THREADS), 0, stream_, dd);
            HIP_OK(hipGetLastError());
            prof_end(2, e0);
        }
    }

    void gather(const std::vector<GatherDesc>& ds) override {
        small<GatherDesc>(ds, k_gather, [](const GatherDesc& g) -> int64_t { return (int64_t)g.rows * g.cols; });
    }
    void fill(const std::vector<FillDesc>& ds) override {
        small<FillDesc>(ds, k_fill, [](const FillDesc& f) -> int64_t {
            return f.dcol ? (int64_t)f.rows : (int64_t)f.rows * f.cols;
        });
    }
    void lists(const std::vector<ListDesc>& ds) override {
        small<ListDesc>(ds, k_lists, [](const ListDesc& l) -> int64_t { return std::max(l.npick, l.nkeep); });
    }
    void sort(const std::vector<SortDesc>& ds) override {
        small<SortDesc>(ds, k_sort, [](const SortDesc& s) -> int64_t { return (int64_t)s.n; });
    }

    int64_t count_out_of_range(const uint8_t* A, int64_t m, int64_t n, int64_t lda, int32_t p) override {
        HIP_OK(hipMemsetAsync(counter_, 0, 8, stream_));
        int64_t total = m * n;
        int64_t bx = std::min<int64_t>((total + SMALL_THREADS - 1) / SMALL_THREADS, 8192);
        hipLaunchKernelGGL(k_range, dim3((unsigned)std::max<int64_t>(bx, 1)), dim3(SMALL_THREADS), 0, stream_, A, m,
                           n, lda, p, (unsigned long long*)counter_);
        HIP_OK(hipGetLastError());
        unsigned long long bad = 0;
        download(&bad, counter_, 8);
        return err_ ? -1 : (int64_t)bad;
    }

    void set_profile(bool on) override { prof_ = on; }
    Profile take_profile() override {
        Profile pr;
        HIP_OK(hipStreamSynchronize(stream_));
        for (auto& ev : evs_) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
                pr.ms[ev.kind] += ms;
                pr.launches[ev.kind] += 1;
            }
            pool_.push_back(ev.a);
            pool_.push_back(ev.b);
        }
        evs_.clear();
        return pr;
    }

private:
    struct Ev { hipEvent_t a, b; int kind; };
    hipEvent_t new_event() {
        if (!pool_.empty()) {
            hipEvent_t e = pool_.back();
            pool_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        HIP_OK(hipEventCreate(&e));
        return e;
    }
    hipEvent_t prof_begin() {
        if (!prof_) return nullptr;
        hipEvent_t e = new_event();
        HIP_OK(hipEventRecord(e, stream_));
        return e;
    }
    void prof_end(int kind, hipEvent_t a) {
        if (!prof_ || !a) return;
        hipEvent_t b = new_event();
        HIP_OK(hipEventRecord(b, stream_));
        evs_.push_back({a, b, kind});
    }

    void note_error(hipError_t e, const char* what) {
        if (!err_) {
            err_ = 6;
            fprintf(stderr, "gfech: %s failed: %s\n", what, hipGetErrorString(e));
        }
    }

    // copy host bytes into the pinned ring; returns the pinned address
    void* stage(const void* src, size_t bytes) {
        size_t need = (bytes + 255) & ~(size_t)255;
        if (ring_off_ + need > kRing) {
            HIP_OK(hipStreamSynchronize(stream_));   // earlier copies out of the ring are done
            ring_off_ = 0;
        }
        void* h = (char*)ring_host_ + ring_off_;
        memcpy(h, src, bytes);
        ring_off_ += need;
        return h;
    }
    // stage descriptors and copy them into the device ring at the same offset
    void* put(const void* src, size_t bytes) {
        void* h = stage(src, bytes);
        size_t off = (char*)h - (char*)ring_host_;
        void* d = (char*)ring_dev_ + off;
        HIP_OK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, stream_));
        return d;
    }

    hipStream_t stream_ = nullptr;
    void* ring_host_ = nullptr;
    void* ring_dev_ = nullptr;
    size_t ring_off_ = 0;
    void* counter_ = nullptr;
    int err_ = 0;
    int num_cu_ = 0;
    bool prof_ = false;
    std::vector<Ev> evs_;
    std::vector<hipEvent_t> pool_;
    std::map<void*, size_t> sizes_;
    std::multimap<size_t, void*> free_;
};

}  // namespace

Backend* backend_instance(std::string* err) {
    static std::mutex mu;
    static HipBackend* be = nullptr;
    static std::string init_err;
    static bool tried = false;
    std::lock_guard<std::mutex> lk(mu);
    if (!tried) {
        tried = true;
        HipBackend* b = new HipBackend();
        if (b->init(&init_err)) be = b;
        else delete b;
    }
    if (!be && err) *err = init_err;
    return be;
}

}  // namespace gfech
