// HIP backend for gfx950 (MI355X): the kernels behind the planner's grouped
// jobs, and the device-memory / stream plumbing.
//
//  - k_gemm_modp   MAD / MUL mod p (the O(n^3) work of UpdateRow,
//                  UpdateRowTrafo, ClearDown and ClearUp) on int8 MFMA
//                  (v_mfma_i32_32x32x32_i8) with int32 accumulation; one
//                  launch runs every descriptor of a phase.
//  - k_ech         ECH (Remark 2.3): one workgroup per block.
//  - k_gather, k_fill, k_lists, k_sort, k_range: extracts, riffles and the
//                  index-list jobs (HBM-bound).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "backend.h"

namespace gfech {
namespace {

// ============================================================================ memory helpers

// Accesses through pointers taken from descriptors in memory would otherwise
// compile to flat instructions, whose completion also gates LDS waits; these
// make them global (address space 1) loads and stores.
#define GPTR(T, p) ((const __attribute__((address_space(1))) T*)(p))
#define GPTRW(T, p) ((__attribute__((address_space(1))) T*)(p))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T gload(const void* p) { return *GPTR(T, p); }
template <>
__device__ __forceinline__ uint4 gload<uint4>(const void* p) {
    const u32x4 v = *GPTR(u32x4, p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ uint2 gload<uint2>(const void* p) {
    const u32x2 v = *GPTR(u32x2, p);
    return make_uint2(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void gstore(void* p, T v) { *GPTRW(T, p) = v; }
template <>
__device__ __forceinline__ void gstore<uint4>(void* p, uint4 v) { *GPTRW(u32x4, p) = u32x4{v.x, v.y, v.z, v.w}; }

// ============================================================================ field helpers

// x mod p for 0 <= x < 2^24, p <= 251: q = floor(x * floor(2^24 / p) / 2^24) is
// floor(x / p) or one less, so one conditional subtraction finishes.
__device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t p, uint32_t minv) {
    uint32_t q = __umulhi(x << 8, minv);
    uint32_t r = x - __umul24(q, p);
    return r >= p ? r - p : r;
}

// a + b * c for b, c < 2^24 (one full-rate v_mad_u32_u24)
__device__ __forceinline__ uint32_t mad24(uint32_t b, uint32_t c, uint32_t a) { return __umul24(b, c) + a; }

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

// ============================================================================ descriptor sources
//
// Every kernel reads its job descriptors through a source: a few of them
// travel by value in the kernel arguments (no upload before the launch),
// larger sets are uploaded and read through a pointer.  Indices are uniform
// across the workgroup.
template <typename D, int CAP>
struct DescArg {
    D d[CAP];
    __device__ __forceinline__ D get(int i) const { return d[i]; }
};
template <typename D>
struct DescPtr {
    const D* p;
    __device__ __forceinline__ D get(int i) const { return p[i]; }
};

// f(std::integral_constant<int, K>) for K = K0 .. N - 1, unrolled at compile time
template <int K0, int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
    if constexpr (K0 < N) {
        f(std::integral_constant<int, K0>{});
        static_for<K0 + 1, N>(f);
    }
}

// ============================================================================ GEMM mod p
//
// Workgroup tile TM x TN of D (TN = 128 or 256, see GemmCfg), 2 x (TN / 64)
// waves, each wave 128 x 64 as 4 x 2 blocks of v_mfma_i32_32x32x32_i8 (on
// this chip it retires half again as
// many products per cycle as the 16 x 16 x 64 form).  The MFMA is issued with
// the operands swapped (the B tile as the first operand) so that a lane's
// results come in runs of four consecutive columns of one row of D: the
// epilogue reduces, packs and stores each run as one dword.  K advances in
// steps of TK, two MFMA k-steps of 32 each.  A is kept [m][k]
// in LDS, 64-byte rows, the 16-byte chunk c of row m at position
// c ^ ((m >> 2) & 3), so the 16 lanes reading one chunk of 16 rows hit 16
// different bank groups.  B is kept as it is stored, [k][n], the 16-byte
// chunk c of row k at position c ^ s(k) (GemmCfg::bswz: s(k) = 2 (k & 7) in
// the 256-column tile, whose rows span all 64 banks, so that the two groups
// of 16 lanes reading chunks 2m and 2m + 1 of the same 8 rows use disjoint
// banks; k & 7 in the 128-column tile); the MFMA wants 16 consecutive k
// of one column per lane, which ds_read_b64_tr_b8 delivers: within each group
// of 16 lanes, lane pairs (2t, 2t + 1) address the two halves of a 16-byte
// row t (t < 8), and lane c of the group receives byte c of each of the 8
// rows.
//
// Interior tiles with unpermuted, 16-byte aligned operands over p <= 127
// stream both tiles straight into LDS (global_load_lds_dwordx4: lane l of a
// wave writes the 16 bytes at the wave's LDS base + 16 l, from any address it
// chooses) through three stages (four for the wide tile), that many steps
// less one ahead of the MFMAs.  The other tiles go through registers, one
// step ahead, in two of the stages.
//
// Exactness: residues of p <= 127 are used as they are, residues of p > 127
// are centred (x >= 128 becomes x - p), so every product is an int8 x int8
// product; |sum| <= K * 127^2 < 2^30 for K <= 65536.  When the sums are small
// (p <= 127 and K (p - 1)^2 + p - 1 < 2^22) the epilogue reduces them with a
// float quotient estimate (mod22), otherwise with a Barrett step (ModP).

constexpr int TM = 256;          // rows of D per workgroup tile
constexpr int TK = 64;           // reduction depth per LDS stage
constexpr int GEMM_A_STAGE = TM * TK;                    // bytes of one A tile

// The two tile widths: WN = 4 wave columns (tile 256 x 256, 8 waves, four
// stages, one workgroup per compute unit), the one used, or WN = 2 (tile
// 256 x 128, 4 waves, three stages, two workgroups per compute unit): the
// same waves per SIMD, and the wide tile moves a third fewer operand bytes
// per multiply-add.
template <int WN>
struct GemmCfg {
    static constexpr int TN = 64 * WN;                  // columns of D per workgroup tile
    static constexpr int WAVES = 2 * WN;                // 2 x WN waves, each 128 x 64
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int BCH = TN / 16;                 // 16-byte chunks per B row
    static constexpr int STAGE = GEMM_A_STAGE + TK * TN;   // A tile, then B tile
    static constexpr int STAGES = WN == 2 ? 3 : 4;   // five for the wide tile measured no faster
    static constexpr int OCC = WN == 2 ? 2 : 1;         // workgroups per compute unit
    static constexpr int A_PIECES = GEMM_A_STAGE / 1024 / WAVES;   // 1 KB pieces per wave and stage
    static constexpr int B_PIECES = TK * TN / 1024 / WAVES;
    static constexpr int RPS = STAGE / TN;              // rows of a C tile one stage holds
    static constexpr int NA = 4 * TM / THREADS;         // A chunks per thread (register path)
    static_assert(A_PIECES >= 1 && B_PIECES >= 1 && TM * TN / 1024 / WAVES == 8, "tile layout");
    static constexpr size_t lds_bytes() { return (size_t)STAGES * STAGE; }
    // position offset of the 16-byte chunks of B row k (chunk c at c ^ bswz(k))
    static __device__ __forceinline__ int bswz(int k) { return BCH == 16 ? (k & 7) << 1 : k & 7; }
};
constexpr int TN = 128;          // the narrow tile's width (host-side tile counts use GemmCfg)

// LDS byte offset of 16-byte chunk c (< 4) of row m of an A tile
__device__ __forceinline__ int a_chunk_pos(int m, int c) { return m * TK + ((c ^ ((m >> 2) & 3)) << 4); }

typedef int v4i __attribute__((ext_vector_type(4)));

struct GemmTileMap {           // per-descriptor tile grid, device side
    int32_t tiles_n;           // tiles along N
    int32_t first_tile;        // prefix sum of tiles
};

// MAD descriptors with their tile grids: by value (up to GEMM_ARG_CAP) or
// through pointers into one uploaded block
constexpr int GEMM_ARG_CAP = 32;
struct GemmArgSrc {
    int n;
    int group;                 // tile rows per group of the tile order (see k_gemm_modp)
    GemmTileMap m[GEMM_ARG_CAP];
    GemmDesc d[GEMM_ARG_CAP];
    __device__ __forceinline__ int count() const { return n; }
    __device__ __forceinline__ GemmTileMap map(int i) const { return m[i]; }
    __device__ __forceinline__ GemmDesc get(int i) const { return d[i]; }
    // the descriptor that owns `tile`: the last one whose first tile is at or
    // before it (first tiles ascend, the first is 0), counted over every
    // entry at once rather than by a chain of dependent loads
    __device__ __forceinline__ int find(int tile) const {
        int c = 0;
#pragma unroll
        for (int i = 1; i < GEMM_ARG_CAP; ++i) c += (i < n && m[i].first_tile <= tile) ? 1 : 0;
        return c;
    }
};
struct GemmPtrSrc {
    int n;
    int group;
    const GemmTileMap* m;
    const GemmDesc* d;
    __device__ __forceinline__ int count() const { return n; }
    __device__ __forceinline__ GemmTileMap map(int i) const { return m[i]; }
    __device__ __forceinline__ GemmDesc get(int i) const { return d[i]; }
    // as GemmArgSrc::find; each lane of the wave tests entries lane, lane + 64, ...
    __device__ __forceinline__ int find(int tile) const {
        const int lane = (int)(threadIdx.x & 63);
        int c = 0;
        for (int b = 0; b < n; b += 256) {
            bool le[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = b + 64 * u + lane;
                le[u] = i < n && m[i].first_tile <= tile;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) c += __popcll(__ballot(le[u]));
        }
        return c - 1;
    }
};

// v mod p for 0 <= v < 2^22.  With inv = fl(1/p), fl(v * inv) differs from
// v / p by less than 0.51 / p, so its integer part q is floor(v / p) or one
// less, and r = v - q p lies in [0, 2p): one conditional subtraction (as an
// unsigned min: r - p wraps around when r < p) finishes.
__device__ __forceinline__ uint32_t mod22(uint32_t v, float inv, uint32_t p) {
    const int q = (int)((float)v * inv);
    const uint32_t r = (uint32_t)(__mul24(q, -(int)p) + (int)v);   // one 24-bit multiply-add
    return min(r, r - p);
}

// 16 bytes starting at any byte address p, of which `rem` (>= 1) are valid.
// Rows with at least 20 valid bytes left are read as aligned dwords and
// realigned (every byte read lies inside the row); shorter tails are read byte
// by byte, so nothing past the last valid byte is ever touched.
__device__ __forceinline__ uint4 load16_lim(const uint8_t* p, int rem) {
    if (rem >= 20) {
        uintptr_t a = (uintptr_t)p;
        const uint32_t* q = (const uint32_t*)(a & ~(uintptr_t)3);
        uint32_t sh = (uint32_t)(a & 3);
        uint32_t w0 = gload<uint32_t>(q), w1 = gload<uint32_t>(q + 1), w2 = gload<uint32_t>(q + 2),
                 w3 = gload<uint32_t>(q + 3);
        if (sh == 0) return make_uint4(w0, w1, w2, w3);
        uint32_t w4 = gload<uint32_t>(q + 4);
        return make_uint4(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
                          __builtin_amdgcn_alignbyte(w3, w2, sh), __builtin_amdgcn_alignbyte(w4, w3, sh));
    }
    uint32_t w[4] = {0, 0, 0, 0};
    int n = rem < 16 ? rem : 16;
    for (int b = 0; b < n; ++b) w[b >> 2] |= (uint32_t)gload<uint8_t>(p + b) << (8 * (b & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}


// 4 bytes starting at p, `rem` (>= 1) valid
__device__ __forceinline__ uint32_t load4_lim(const uint8_t* p, int rem) {
    uintptr_t a = (uintptr_t)p;
    if ((a & 3) == 0 && rem >= 4) return gload<uint32_t>(p);
    uint32_t w = 0;
    int n = rem < 4 ? rem : 4;
    for (int b = 0; b < n; ++b) w |= (uint32_t)gload<uint8_t>(p + b) << (8 * b);
    return w;
}

// residues of p > 127 become signed int8 values x - p for x >= 128: add 256 - p to those bytes
__device__ __forceinline__ uint32_t centre(uint32_t w, uint32_t adj) {
    uint32_t hi = (w >> 7) & 0x01010101u;
    return w + hi * adj;
}


// 16 bytes at p for an interior tile (no bounds checks): one vector load
// when p is 16-byte aligned, else aligned dwords realigned with alignbyte
// (then up to 3 bytes past the chunk are read; the caller keeps them inside
// the row)
__device__ __forceinline__ uint4 load16_any(const uint8_t* p) {
    const uintptr_t a = (uintptr_t)p;
    if ((a & 15) == 0) return gload<uint4>(p);
    const uint32_t* q = (const uint32_t*)(a & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(a & 3);
    const uint32_t w0 = gload<uint32_t>(q), w1 = gload<uint32_t>(q + 1), w2 = gload<uint32_t>(q + 2),
                   w3 = gload<uint32_t>(q + 3);
    if (sh == 0) return make_uint4(w0, w1, w2, w3);
    const uint32_t w4 = gload<uint32_t>(q + 4);
    return make_uint4(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
                      __builtin_amdgcn_alignbyte(w3, w2, sh), __builtin_amdgcn_alignbyte(w4, w3, sh));
}

template <int WN>
struct GemmRegs {
    uint4 a[GemmCfg<WN>::NA];   // A: 16-byte chunks tid, tid + THREADS, .. (row c / 4, chunk c % 4)
    uint4 b[2];                 // B: k-rows tid / BCH and that + 32, 16 columns from 16 (tid % BCH)
};

// Interior tiles (FAST): no bounds checks, so the loads stay in flight while
// the MFMAs of the current step run.  Otherwise every chunk is checked.
template <bool FAST, int WN>
__device__ __forceinline__ void gemm_load(const GemmDesc& g, int m0, int n0, int k0, int tid, uint32_t adj,
                                          GemmRegs<WN>& R) {
    using GC = GemmCfg<WN>;
    constexpr int NA = GC::NA, GEMM_THREADS = GC::THREADS;
    const int kr = tid / GC::BCH, cb = (tid % GC::BCH) * 16;
    if (FAST) {
        int64_t br[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) br[h] = g.brow ? gload<int32_t>(g.brow + k0 + kr + 32 * h) : k0 + kr + 32 * h;
#pragma unroll
        for (int s = 0; s < NA; ++s) {
            const int c = tid + s * GEMM_THREADS;
            R.a[s] = gload<uint4>(g.A + (int64_t)(m0 + (c >> 2)) * g.lda + k0 + (c & 3) * 16);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) R.b[h] = load16_any(g.B + br[h] * g.ldb + n0 + cb);
        if (adj) {
#pragma unroll
            for (int s = 0; s < NA; ++s) {
                R.a[s].x = centre(R.a[s].x, adj); R.a[s].y = centre(R.a[s].y, adj);
                R.a[s].z = centre(R.a[s].z, adj); R.a[s].w = centre(R.a[s].w, adj);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                R.b[h].x = centre(R.b[h].x, adj); R.b[h].y = centre(R.b[h].y, adj);
                R.b[h].z = centre(R.b[h].z, adj); R.b[h].w = centre(R.b[h].w, adj);
            }
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < NA; ++s) {
        const int c = tid + s * GEMM_THREADS;
        const int row = c >> 2, kc = (c & 3) * 16;
        const int gr = m0 + row, gk = k0 + kc;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gr < g.M && gk < g.K) {
            v = load16_lim(g.A + (int64_t)gr * g.lda + gk, g.K - gk);
            if (adj) { v.x = centre(v.x, adj); v.y = centre(v.y, adj); v.z = centre(v.z, adj); v.w = centre(v.w, adj); }
        }
        R.a[s] = v;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int gk = k0 + kr + 32 * h, gn = n0 + cb;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gk < g.K && gn < g.N) {
            const int64_t br = g.brow ? gload<int32_t>(g.brow + gk) : gk;
            v = load16_lim(g.B + br * g.ldb + gn, g.N - gn);
            if (adj) { v.x = centre(v.x, adj); v.y = centre(v.y, adj); v.z = centre(v.z, adj); v.w = centre(v.w, adj); }
        }
        R.b[h] = v;
    }
}

template <int WN>
__device__ __forceinline__ void gemm_store_lds(const GemmRegs<WN>& R, uint8_t* As, uint8_t* Bs, int tid) {
    using GC = GemmCfg<WN>;
#pragma unroll
    for (int s = 0; s < GC::NA; ++s) {
        const int c = tid + s * GC::THREADS;
        *(uint4*)(As + a_chunk_pos(c >> 2, c & 3)) = R.a[s];
    }
    // k-rows kr and kr + 32 share the swizzle
    const int kr = tid / GC::BCH, pos = ((tid % GC::BCH) ^ GC::bswz(kr)) << 4;
    *(uint4*)(Bs + kr * GC::TN + pos) = R.b[0];
    *(uint4*)(Bs + (kr + 32) * GC::TN + pos) = R.b[1];
}

// 16 bytes from global address g into LDS at (wave-uniform) lds_base + 16 * lane.
// Written as assembly so that the compiler does not guard later LDS reads
// with a wait for every load in flight; the kernel waits itself (vm_wait).
__device__ __forceinline__ void dma16(const void* g, uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds_base) : "memory");
}
// the same with the non-temporal hint, for data no other tile reads
__device__ __forceinline__ void dma16_nt(const void* g, uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt" ::"v"(g), "s"(lds_base) : "memory");
}
// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt left at their maximum)
template <int N>
__device__ __forceinline__ void vm_wait() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

typedef int v2i __attribute__((ext_vector_type(2)));
// 8 bytes per lane through ds_read_b64_tr_b8 (see the comment at the top of this section)
__device__ __forceinline__ v2i lds_read_tr8(const uint8_t* p) {
    return __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i*)(p));
}

typedef int v16i __attribute__((ext_vector_type(16)));

template <int WN, class Src>
__global__ void __launch_bounds__(GemmCfg<WN>::THREADS, GemmCfg<WN>::OCC) k_gemm_modp(Src src) {
    using GC = GemmCfg<WN>;
    constexpr int TN = GC::TN, GEMM_THREADS = GC::THREADS, GEMM_STAGE = GC::STAGE, NS = GC::STAGES;
    constexpr int PCS = GC::A_PIECES + GC::B_PIECES;   // 1 KB pieces per wave and stage
    constexpr int IM = 4;                 // 32-row MFMA blocks per wave
    constexpr int JN = 2;                 // 32-column MFMA blocks per wave
    extern __shared__ __attribute__((aligned(16))) uint8_t gsm[];
    // stage s: A tile at As(s) ([m][k], swizzled), B tile at Bs(s) ([k][n], swizzled)
    const auto As = [](int s) { return gsm + s * GEMM_STAGE; };
    const auto Bs = [](int s) { return gsm + s * GEMM_STAGE + GEMM_A_STAGE; };

    // Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b mod 8),
    // each with its own L2.  Tiles are renumbered so that XCD x takes one
    // contiguous range of them: the tiles of one descriptor, which share A
    // panels, then mostly run on the same XCD.
    const int tile = [] {
        const int nt = (int)gridDim.x, b = (int)blockIdx.x;
        const int q = nt >> 3, rem = nt & 7, x = b & 7;
        return x * q + (x < rem ? x : rem) + (b >> 3);
    }();
    const int lo = src.find(tile);
    const GemmDesc g = src.get(lo);
    const GemmTileMap gm = src.map(lo);
    const int local = tile - gm.first_tile;
    const int tn = gm.tiles_n;
    // Tile order inside a descriptor: groups of `group` tile rows, each group
    // column by column, so consecutive tiles share their B panel (and a group's
    // A panels) while they are in the XCD's L2; group 1 is row by row.
    int m0, n0;
    {
        const int tm = (g.M + TM - 1) / TM;
        const int G = src.group;
        const int grp = local / (G * tn);
        const int rows = min(G, tm - grp * G);
        const int idx = local - grp * G * tn;
        m0 = (grp * G + idx % rows) * TM;
        n0 = (idx / rows) * TN;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = (wave / WN) * 128;     // wave's 128 x 64 sub-tile
    const int wn = (wave % WN) * 64;
    const uint32_t p = (uint32_t)g.p;
    const uint32_t adj = p > 127 ? 256u - p : 0u;

    v16i acc[IM][JN];
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;

    const int nk = (g.K + TK - 1) / TK;
    // steps that may use the unchecked loads: the whole tile inside D, A rows
    // 16-byte aligned, and B rows either aligned for the vector load or with
    // 3 spare columns after the tile for the realigning read
    const bool b_aligned = (((uintptr_t)g.B | (uintptr_t)g.ldb) & 15) == 0;
    const bool a_aligned = ((uintptr_t)g.A & 15) == 0 && (g.lda & 15) == 0;
    const bool fast = m0 + TM <= g.M && n0 + TN <= g.N && a_aligned && (b_aligned || n0 + TN + 3 <= g.N);
    const int nk_fast = fast ? g.K / TK : 0;
    // The streamed path also takes edge tiles: A rows past M read row M - 1,
    // B and C chunks past N read column 0, so every read stays inside the
    // operands, and what they contribute lands in rows or columns of D that
    // are not stored.  A chunk across N reads up to 15 bytes past it: only
    // when N is a multiple of 16 (no such chunk) or the rows are padded.
    // Gathered B rows (brow) stream when K is at most 4 steps: the row numbers
    // of every step are loaded before the first transfer.
    const bool stream = a_aligned && b_aligned && adj == 0 && g.K >= TK && (!g.brow || g.K <= 4 * TK) &&
                        (n0 + TN <= g.N || (g.N & 15) == 0 || (g.flags & kGemmRowsPadded));
    const int nk_str = stream ? g.K / TK : 0;
    const int r16 = lane & 15;
    const int r32 = lane & 31;
    const int kh = lane >> 5;

    // The operands of one half of a K step (32 of its 64 k) on LDS stage st:
    // B operand of block j: lane 32 kh + c gets column wn + 32 j + c and
    // k = 32 h + 16 kh .. + 15; its group of 16 lanes reads rows k0 + t and
    // k0 + 8 + t (t = r16 / 2, whose swizzle is bswz(t)) of the 16-column chunk
    // (wn + 32 j) / 16 + (c >= 16) at half r16 & 1.  A operand of block i:
    // row wm + 32 i + r32, the same 16 k (chunk 2 h + kh).
    struct Half { v4i a[IM]; v4i b[JN]; };
    const auto read_half = [&](int st, int h, Half& f) {
        const int k0 = 32 * h + 16 * kh, t = r16 >> 1;
#pragma unroll
        for (int j = 0; j < JN; ++j) {
            const int ch = (wn >> 4) + 2 * j + ((lane >> 4) & 1);
            const uint8_t* rp = Bs(st) + (k0 + t) * TN + ((ch ^ GC::bswz(t)) << 4) + ((r16 & 1) << 3);
            const v2i lo2 = lds_read_tr8(rp), hi2 = lds_read_tr8(rp + 8 * TN);
            f.b[j] = v4i{lo2.x, lo2.y, hi2.x, hi2.y};
        }
#pragma unroll
        for (int i = 0; i < IM; ++i) f.a[i] = *(const v4i*)(As(st) + a_chunk_pos(wm + i * 32 + r32, 2 * h + kh));
    };
    // the 4 x 2 MFMAs 32 x 32 x 32 of one half
    const auto mma_half = [&](const Half& f) {
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.b[j], f.a[i], acc[i][j], 0, 0, 0);
    };
    // the same, with `between(m)` called after MFMA m (m < 8)
    const auto mma_half_with = [&](const Half& f, auto between) {
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.b[j], f.a[i], acc[i][j], 0, 0, 0);
                between(i * JN + j);
            }
    };
    // one K step on LDS stage st, operands read as it goes
    const auto mma_step = [&](int st) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            Half f;
            read_half(st, h, f);
            mma_half(f);
        }
    };

    GemmRegs<WN> R;
    // LDS epilogue: the C tile arrives in LDS during the last step, D leaves
    // through LDS as whole 16-byte row chunks.  Stage of the last step, or -1.
    int epi_st = -1;
    const bool al16_c = !g.C || (!g.crow && ((((uintptr_t)g.C) | (uintptr_t)g.ldc) & 15) == 0);
    const bool al16_d = ((((uintptr_t)g.D) | (uintptr_t)g.ldd) & 15) == 0;
    if (stream) {
        const bool lds_epi = al16_c && al16_d;
        // ---- streamed into LDS, NS - 1 steps ahead.  Per wave and stage:
        // A_PIECES 1 KB pieces of the A tile (chunk P = piece * 64 + lane is row
        // P / 4, position P % 4) and B_PIECES of the B tile (chunk P is k-row
        // P / BCH, position P % BCH), each lane loading the global chunk its LDS
        // position holds.
        const uint32_t lds0 = (uint32_t)(uintptr_t)gsm;
        const uint8_t* asrc[GC::A_PIECES];
        const uint8_t* bsrc[2];
#pragma unroll
        for (int t = 0; t < GC::A_PIECES; ++t) {
            const int P = (wave * GC::A_PIECES + t) * 64 + lane, row = P >> 2, pos = P & 3;
            asrc[t] = g.A + (int64_t)min(m0 + row, g.M - 1) * g.lda + ((pos ^ ((row >> 2) & 3)) << 4);
        }
        // B row of k-row kr of step s: brow[s * TK + kr] when gathered (bix[s][t]
        // for piece t, loaded now and waited for here, so that no load into a
        // register is in flight once the transfers start), else s * TK + kr
        int bix[4][2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int P = (wave * GC::B_PIECES + t) * 64 + lane, kr = P / GC::BCH, pos = P % GC::BCH;
            const int col = n0 + ((pos ^ GC::bswz(kr)) << 4);
            bsrc[t] = g.B + (col < g.N ? col : 0);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                bix[s4][t] = g.brow ? (s4 < nk_str ? gload<int32_t>(g.brow + s4 * TK + kr) : 0) : s4 * TK + kr;
        }
        if (g.brow) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) asm volatile("" ::"v"(bix[s4][0]), "v"(bix[s4][1]));
        }
        // A descriptor of one tile row reads each B panel once (the products
        // of a Step-1 layer): those transfers carry the non-temporal hint, so
        // that the panels do not displace the A panels the row's tiles share
        // from the L2.  (With several tile rows B is shared: the hint would
        // cost the reuse.  Measured: the isolated layer launch 0.486 ->
        // 0.457 ms with the hint on B; the largest ClearUp launch 5.27 ->
        // 6.18 ms if its B carried it too.)  C is read once by every tile.
        const bool b_once = g.M <= TM;
        // ungathered B: piece t of step ks reads from bbase[t] + ks TK ldb
        const uint8_t* bbase[2] = {bsrc[0] + (int64_t)bix[0][0] * g.ldb, bsrc[1] + (int64_t)bix[0][1] * g.ldb};
        const int64_t bstep = (int64_t)TK * g.ldb;
        // piece q (< PCS) of step ks into stage st: the A pieces, then the B pieces
        const auto piece = [&](int ks, int st, int q) {
            const uint32_t base = lds0 + (uint32_t)(st * GEMM_STAGE);
            if (q < GC::A_PIECES) {
                dma16(asrc[q] + (int64_t)ks * TK, base + (uint32_t)((wave * GC::A_PIECES + q) * 1024));
            } else {
                const int t = q - GC::A_PIECES;
                const uint8_t* src = g.brow ? bsrc[t] + (int64_t)(ks == 0 ? bix[0][t] : ks == 1 ? bix[1][t] : ks == 2 ? bix[2][t] : bix[3][t]) * g.ldb
                                            : bbase[t] + ks * bstep;
                const uint32_t dst = base + (uint32_t)(GEMM_A_STAGE + (wave * GC::B_PIECES + t) * 1024);
                if (b_once) dma16_nt(src, dst);
                else dma16(src, dst);
            }
        };
        const auto issue = [&](int ks, int st) {
#pragma unroll
            for (int q = 0; q < PCS; ++q) piece(ks, st, q);
        };
#pragma unroll
        for (int s0 = 0; s0 < NS; ++s0)
            if (s0 < nk_str) issue(s0, s0);
        // the C tile of the last step goes to the next two stages (rows
        // 0 .. RPS - 1 in the next, the rest in the one after) while its MFMAs
        // run; 8 pieces of 1 KB per wave, each 1024 / TN whole rows
        const auto fetch_c = [&](int st) {
            epi_st = st;
            if (!g.C) return;
            const uint32_t s1 = lds0 + (uint32_t)(((st + 1) % NS) * GEMM_STAGE);
            const uint32_t s2 = lds0 + (uint32_t)(((st + 2) % NS) * GEMM_STAGE);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int r0 = (wave * 8 + t) * (1024 / TN), row = r0 + lane / GC::BCH, pos = lane % GC::BCH;
                const uint32_t base = r0 < GC::RPS ? s1 + (uint32_t)(r0 * TN) : s2 + (uint32_t)((r0 - GC::RPS) * TN);
                const int col = n0 + ((pos ^ ((row >> 1) & 7)) << 4);
                dma16_nt(g.C + (int64_t)min(m0 + row, g.M - 1) * g.ldc + (col < g.N ? col : 0),
                         __builtin_amdgcn_readfirstlane(base));
            }
        };
        // this wave's pieces of step `next` have landed, `later` steps after it
        // being in flight (PCS pieces each)
        const auto wait_step = [&](int later) {
            if (later >= 3) vm_wait<3 * PCS>();
            else if (later == 2) vm_wait<2 * PCS>();
            else if (later == 1) vm_wait<PCS>();
            else vm_wait<0>();
        };
        // No load into registers may sit inside this loop: the compiler would
        // guard every use of a register it writes with a wait for all loads in
        // flight, the DMA of the next steps included.
        //
        // Step ks runs its first half's MFMAs on operands read before, then
        // waits for step ks + 1 and meets the other waves at the barrier: by
        // then every wave has read all of step ks into registers, so its stage
        // takes step ks + NS, and step ks + 1 is visible.  The first half of
        // step ks + 1 is read while the second half's MFMAs of step ks run,
        // and its second half after them: the reads' latency stays off the
        // matrix cores' path, and the barrier falls between two groups of
        // MFMAs rather than before a group's operands are read.
        wait_step(min(NS - 1, nk_str - 1));
        __syncthreads();
        Half f0, f1;
        read_half(0, 0, f0);
        read_half(0, 1, f1);
        // The transfers of step ks + NS go out one or two at a time between
        // the second half's MFMAs: a wave whose transfer waits for the
        // memory pipeline's queue cannot issue anything after it.  (The last
        // step is peeled off, and the steps that issue no transfer get a loop
        // of their own, so that the loops' reads are unconditional and the
        // compiler's waits count them exactly.)
        int st = 0;
        const auto body = [&](int ks, auto dma) {
            const int nst = st + 1 == NS ? 0 : st + 1;
            mma_half(f0);
            wait_step(min(NS - 2, nk_str - 2 - ks));
            __syncthreads();
            read_half(nst, 0, f0);
            if constexpr (decltype(dma)::value) {
                mma_half_with(f1, [&](int m) {
                    static_for<0, PCS>([&](auto q) {
                        if (q * 8 / PCS == m) {
                            __builtin_amdgcn_sched_barrier(0);
                            piece(ks + NS, st, q);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    });
                });
            } else {
                mma_half(f1);
            }
            read_half(nst, 1, f1);
            st = nst;
        };
        int ks = 0;
        for (; ks + NS < nk_str; ++ks) body(ks, std::true_type{});
        for (; ks + 1 < nk_str; ++ks) body(ks, std::false_type{});
        mma_half(f0);
        if (nk == nk_str && lds_epi) fetch_c(st);
        mma_half(f1);
        st = st + 1 == NS ? 0 : st + 1;
        if (nk > nk_str) {
            // the K tail (one step) through registers: its stage was last read
            // by step nk_str - NS, which every wave has passed
            gemm_load<false>(g, m0, n0, nk_str * TK, tid, adj, R);
            gemm_store_lds(R, As(st), Bs(st), tid);
            __syncthreads();
            if (lds_epi) fetch_c(st);
            mma_step(st);
        }
    } else {
        // ---- through registers, one step ahead, stages 0 and 1
        if (nk > 0) {
            if (nk_fast > 0) gemm_load<true>(g, m0, n0, 0, tid, adj, R);
            else gemm_load<false>(g, m0, n0, 0, tid, adj, R);
            gemm_store_lds(R, As(0), Bs(0), tid);
        }
        __syncthreads();
        for (int ks = 0; ks < nk; ++ks) {
            const int st = ks & 1;
            if (ks + 1 < nk_fast) gemm_load<true>(g, m0, n0, (ks + 1) * TK, tid, adj, R);
            else if (ks + 1 < nk) gemm_load<false>(g, m0, n0, (ks + 1) * TK, tid, adj, R);
            mma_step(st);
            if (ks + 1 < nk) gemm_store_lds(R, As(st ^ 1), Bs(st ^ 1), tid);
            __syncthreads();
        }
    }

    // ---- epilogue: D = (Cin + acc) mod p.  Lane holds, for block (i, j) and
    // q < 4, row wm + 32 i + lane % 32 and the four columns
    // wn + 32 j + 8 q + 4 (lane / 32) + e in acc[i][j][4 q + e].
    const auto acc4 = [&](int i, int j, int q) {
        return v4i{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
    };
    const bool small = p <= 127 && (uint64_t)g.K * (p - 1) * (p - 1) + (p - 1) < (1u << 22);
    const float inv = 1.0f / (float)p;
    const ModP mod(p);
    const auto reduce4 = [&](const v4i& a, uint32_t cw) -> uint32_t {
        uint32_t out = 0;
        if (small) {
#pragma unroll
            for (int e = 0; e < 4; ++e) out |= mod22((uint32_t)a[e] + ((cw >> (8 * e)) & 0xffu), inv, p) << (8 * e);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) out |= mod(a[e] + (int)((cw >> (8 * e)) & 0xffu)) << (8 * e);
        }
        return out;
    };
    if (epi_st >= 0) {
        // C tile row m at cl(m), its 16-byte chunk c at position c ^ ((m >> 1) & 7):
        // the 16 lanes reading one chunk of 16 rows hit 16 different bank groups
        uint8_t* const s1 = As((epi_st + 1) % NS);
        uint8_t* const s2 = As((epi_st + 2) % NS);
        const auto cl = [&](int m) { return m < GC::RPS ? s1 + m * TN : s2 + (m - GC::RPS) * TN; };
        vm_wait<0>();
        __syncthreads();
        // each lane reads all its C words, then writes its D words in their
        // place: the reads are in flight together and no write precedes a read
        // it might alias; the uniform choices (C present, reduction) are taken
        // once for the whole tile, not per word
        const auto wp = [&](int i, int j, int q) {
            const int row = wm + i * 32 + r32;
            const int ch = (wn >> 4) + 2 * j + (q >> 1);
            return (uint32_t*)(cl(row) + ((ch ^ ((row >> 1) & 7)) << 4) + (q & 1) * 8 + kh * 4);
        };
        uint32_t cw[IM][JN][4];
        if (g.C) {
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int j = 0; j < JN; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) cw[i][j][q] = *wp(i, j, q);
        } else {
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int j = 0; j < JN; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) cw[i][j][q] = 0;
        }
        if (small) {
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int j = 0; j < JN; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const v4i a = acc4(i, j, q);
                        uint32_t out = 0;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            out |= mod22((uint32_t)a[e] + ((cw[i][j][q] >> (8 * e)) & 0xffu), inv, p) << (8 * e);
                        *wp(i, j, q) = out;
                    }
        } else {
#pragma unroll
            for (int i = 0; i < IM; ++i)
#pragma unroll
                for (int j = 0; j < JN; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const v4i a = acc4(i, j, q);
                        uint32_t out = 0;
#pragma unroll
                        for (int e = 0; e < 4; ++e) out |= mod(a[e] + (int)((cw[i][j][q] >> (8 * e)) & 0xffu)) << (8 * e);
                        *wp(i, j, q) = out;
                    }
        }
        __syncthreads();
        // whole 16-byte chunks of D rows: chunk P = tid + THREADS u is row P / BCH, position P % BCH
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int P = tid + u * GEMM_THREADS, row = P / GC::BCH, pos = P % GC::BCH;
            const uint4 v = *(const uint4*)(cl(row) + pos * 16);
            const int col = n0 + ((pos ^ ((row >> 1) & 7)) << 4);
            if (m0 + row < g.M && col < g.N) {
                uint8_t* dp = g.D + (int64_t)(m0 + row) * g.ldd + col;
                if (col + 16 <= g.N) {
                    gstore<uint4>(dp, v);
                } else {   // the chunk across N
                    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                    for (int b = 0; b < g.N - col; ++b) gstore<uint8_t>(dp + b, (uint8_t)(w[b >> 2] >> (8 * (b & 3))));
                }
            }
        }
        return;
    }
    const bool whole = m0 + TM <= g.M && n0 + TN <= g.N &&
                       ((((uintptr_t)g.D) | (uintptr_t)g.ldd | (uintptr_t)g.C | (uintptr_t)g.ldc) & 3) == 0;
    if (whole) {
        // interior tile with dword-aligned rows: every C word is loaded before any
        // is used, so the loads of the whole tile are in flight together
        uint32_t cw[IM][JN][4];
#pragma unroll
        for (int i = 0; i < IM; ++i) {
            const int row = m0 + wm + i * 32 + r32;
            const uint8_t* cp = g.C ? g.C + (int64_t)(g.crow ? gload<int32_t>(g.crow + row) : row) * g.ldc : nullptr;
#pragma unroll
            for (int j = 0; j < JN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    cw[i][j][q] = cp ? gload<uint32_t>(cp + n0 + wn + j * 32 + q * 8 + kh * 4) : 0u;
        }
#pragma unroll
        for (int i = 0; i < IM; ++i) {
            uint8_t* dp = g.D + (int64_t)(m0 + wm + i * 32 + r32) * g.ldd + n0 + wn + kh * 4;
#pragma unroll
            for (int j = 0; j < JN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) gstore<uint32_t>(dp + j * 32 + q * 8, reduce4(acc4(i, j, q), cw[i][j][q]));
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < IM; ++i) {
        const int row = m0 + wm + i * 32 + r32;
        if (row >= g.M) continue;
        const uint8_t* crow_ptr = g.C ? g.C + (int64_t)(g.crow ? gload<int32_t>(g.crow + row) : row) * g.ldc : nullptr;
        uint8_t* drow_ptr = g.D + (int64_t)row * g.ldd;
#pragma unroll
        for (int jq = 0; jq < JN * 4; ++jq) {
            const int j = jq >> 2, q = jq & 3;
            const int col = n0 + wn + j * 32 + q * 8 + kh * 4;
            if (col >= g.N) continue;
            const int rem = g.N - col;
            const uint32_t cw = crow_ptr ? load4_lim(crow_ptr + col, rem) : 0u;
            const uint32_t out = reduce4(acc4(i, j, q), cw);
            uint8_t* dp = drow_ptr + col;
            if (rem >= 4 && (((uintptr_t)dp) & 3) == 0) {
                gstore<uint32_t>(dp, out);
            } else {
                const int n = rem < 4 ? rem : 4;
                for (int e = 0; e < n; ++e) gstore<uint8_t>(dp + e, (uint8_t)(out >> (8 * e)));
            }
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
template <class Src>
__global__ void __launch_bounds__(ECH_THREADS) k_ech(Src src) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    __shared__ int red[ECH_THREADS / 64];
    __shared__ uint32_t s_scale;
    const EchDesc e = src.get(blockIdx.x);
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
    for (int x = wave; x < rows; x += ECH_THREADS / 64)
        for (int y = lane; y < width; y += 64)
            e.work[(int64_t)x * e.ldw + y] = y < cols ? e.H[(int64_t)x * e.ldh + y] : 0;
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
        for (int y = 0; y < e.qtail; ++y) e.qcol[q + y] = cols + y;
    }
    __syncthreads();
    // Mo[t][u] = T[prow[t]][u];  Ro[t][k] = W[prow[t]][qcol[k]];  Ko[s][u] = T[qrow[s]][u]
    for (int t = wave; t < r; t += ECH_THREADS / 64) {
        for (int u = lane; u < r; u += 64) e.Mo[(int64_t)t * e.ldm + u] = e.work[(int64_t)piv_rows[t] * e.ldw + cols + u];
        for (int k = lane; k < cols - r; k += 64)
            e.Ro[(int64_t)t * e.ldr + k] = e.work[(int64_t)piv_rows[t] * e.ldw + e.qcol[k]];
    }
    for (int s2 = wave; s2 < rows - r; s2 += ECH_THREADS / 64)
        for (int u = lane; u < r; u += 64) e.Ko[(int64_t)s2 * e.ldk + u] = e.work[(int64_t)e.qrow[s2] * e.ldw + cols + u];
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
constexpr int ECH_ARG_CAP = 28;        // descriptors passed by value (28 x 136 bytes)

__host__ __device__ constexpr size_t echp_fixed_lds() {
    return 128 + 2 * 16 * 64 * 4 + 2 * ECHP_MAX_ROWS * 4 + 256 * 4 + 2 * ECHP_MAX_ROWS + VCH * FL_ROW;
}
__host__ __device__ inline size_t echp_lds_bytes(int rows) {
    return echp_fixed_lds() + (size_t)((rows + 15) & ~15) * (FL_ROW + VCH);
}

// (a + b) mod p on four packed residues (both < p <= 251), in 16-bit lanes
__device__ __forceinline__ uint32_t addmod4(uint32_t a, uint32_t b, uint32_t p) {
    const uint32_t k = (0x8000u - p) * 0x00010001u, pp = p * 0x00010001u;
    uint32_t lo = (a & 0x00ff00ffu) + (b & 0x00ff00ffu);
    uint32_t hi = ((a >> 8) & 0x00ff00ffu) + ((b >> 8) & 0x00ff00ffu);
    lo -= ((lo + k) >> 15 & 0x00010001u) * p;
    hi -= ((hi + k) >> 15 & 0x00010001u) * p;
    (void)pp;
    return lo | (hi << 8);
}

template <class Src>
__global__ void __launch_bounds__(512) k_ech_panel(Src src) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const EchDesc e = src.get(blockIdx.x);
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
    uint8_t* St = Fl + rows16 * FL_ROW;                            // [rows16][VCH] staged products

    // invt[v] = -1/v mod p: the multiplier that turns a pivot v into -1
    for (int i = x; i < 256; i += nthr) invt[i] = (i > 0 && (uint32_t)i < p) ? (p - pow_mod_dev((uint32_t)i, p - 2, p)) % p : 0u;
    for (int i = x; i < ECHP_MAX_ROWS; i += nthr) sel[i] = 0;
    for (int i = x; i < 32; i += nthr) cand[i] = 0x7fffffff;
    // W = [H | 0]: 16 bytes per lane where the rows are aligned, bytes otherwise
    {
        const bool vec = ((((uintptr_t)e.H) | ((uintptr_t)e.work) | (uintptr_t)e.ldh | (uintptr_t)e.ldw) & 15) == 0;
        for (int rr = wave; rr < rows; rr += nwaves) {
            const uint8_t* src = e.H + (int64_t)rr * e.ldh;
            uint8_t* dst = e.work + (int64_t)rr * e.ldw;
            if (vec) {
                for (int y = lane * 16; y < width; y += 64 * 16) {
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (y + 16 <= cols) v = gload<uint4>(src + y);
                    else if (y < cols) v = load16_lim(src + y, cols - y);
                    if (y + 16 <= width) gstore<uint4>(dst + y, v);
                    else {
                        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int bb = 0; bb < 16; ++bb)
                            if (y + bb < width) gstore<uint8_t>(dst + y + bb, (uint8_t)(w4[bb >> 2] >> (8 * (bb & 3))));
                    }
                }
            } else {
                for (int y = lane; y < width; y += 64) gstore<uint8_t>(dst + y, y < cols ? gload<uint8_t>(src + y) : 0);
            }
        }
    }
    __syncthreads();
    uint8_t* Wx = e.work + (int64_t)x * e.ldw;

    int r = 0;
    for (int c0 = 0; c0 < cols && r < maxr; c0 += PW) {
        const int wc = min(PW, cols - c0);
        uint32_t reg[PW], F[PW];
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            reg[j] = (x < rows && j < wc) ? gload<uint8_t>(Wx + c0 + j) : 0u;
            F[j] = 0;
        }
        bool mysel = x < rows && sel[x];
        bool mine = false;
        uint32_t myscale = 0;
        int rp = 0;
        // The window reg[0..PW) is a shift register: at step k, reg[0] holds column
        // c0 + k.  A column is final once its step is done (later pivots are zero
        // there), so it rotates to the back; after PW steps reg[j] is column c0 + j
        // again.  Every register index is static, so the loop stays rolled.
#pragma clang loop unroll(disable)
        for (int k = 0; k < PW; ++k) {
            if (k < wc && r + rp < maxr) {
                const uint32_t v = mod_small(reg[0], p, minv);
                reg[0] = v;
                const bool isc = x < rows && !mysel && v != 0;
                const unsigned long long bal = __ballot(isc);
                const int par = k & 1;
                if (bal) {
                    // this wave's first candidate parks its window and transform row
                    // (with a 1 for itself); the wave reduces them
                    const int first = __ffsll((long long)bal) - 1;
                    uint32_t* my = slot + (par * 16 + wave) * 64;
                    if (lane == first) {
                        cand[par * 16 + wave] = x;
                        uint4* my4 = (uint4*)my;
#pragma unroll
                        for (int q = 0; q < PW / 4; ++q)
                            my4[q] = make_uint4(reg[4 * q], reg[4 * q + 1], reg[4 * q + 2], reg[4 * q + 3]);
#pragma unroll
                        for (int q = 0; q < PW / 4; ++q)
                            my4[PW / 4 + q] = make_uint4(4 * q == rp ? 1u : F[4 * q], 4 * q + 1 == rp ? 1u : F[4 * q + 1],
                                                         4 * q + 2 == rp ? 1u : F[4 * q + 2],
                                                         4 * q + 3 == rp ? 1u : F[4 * q + 3]);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    my[lane] = mod_small(my[lane], p, minv);
                } else if (lane == 0) {
                    cand[par * 16 + wave] = 0x7fffffff;
                }
                __syncthreads();
                int best = 0x7fffffff;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int4 c4 = ((const int4*)(cand + par * 16))[q];
                    best = min(best, min(min(c4.x, c4.y), min(c4.z, c4.w)));
                }
                if (best != 0x7fffffff) {
                    const uint32_t* ps = slot + (par * 16 + (best >> 6)) * 64;
                    uint32_t pv[2 * PW];
#pragma unroll
                    for (int q = 0; q < PW / 2; ++q) {
                        const uint4 w4 = ((const uint4*)ps)[q];
                        pv[4 * q] = w4.x; pv[4 * q + 1] = w4.y; pv[4 * q + 2] = w4.z; pv[4 * q + 3] = w4.w;
                    }
                    const uint32_t s = invt[pv[0]];                   // -1 / pivot
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
                        const uint32_t f = mod_small(__umul24(v, s), p, minv);
#pragma unroll
                        for (int j = 1; j < PW; ++j) reg[j] = mad24(f, pv[j], reg[j]);
                        reg[0] = 0;
#pragma unroll
                        for (int t = 0; t < PW; ++t) F[t] = mad24(f, pv[PW + t], F[t]);
                    }
                    ++rp;
                }
            }
            const uint32_t done = reg[0];
#pragma unroll
            for (int j = 0; j + 1 < PW; ++j) reg[j] = reg[j + 1];
            reg[PW - 1] = done;
        }
        // normalise this panel's pivot rows (pivot -> -1) and reduce everything
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            uint32_t a = mod_small(reg[j], p, minv), b = mod_small(F[j], p, minv);
            if (mine) {
                a = mod_small(__umul24(a, myscale), p, minv);
                b = mod_small(__umul24(b, myscale), p, minv);
            }
            reg[j] = a;
            F[j] = b;
        }
        if (x < rows) {
            uint32_t pw[PW / 4], fw[PW / 4];
#pragma unroll
            for (int q = 0; q < PW / 4; ++q) {
                pw[q] = reg[4 * q] | (reg[4 * q + 1] << 8) | (reg[4 * q + 2] << 16) | (reg[4 * q + 3] << 24);
                fw[q] = F[4 * q] | (F[4 * q + 1] << 8) | (F[4 * q + 2] << 16) | (F[4 * q + 3] << 24);
            }
            uint8_t* dp = Wx + c0;
            if (wc == PW && (((uintptr_t)dp) & 15) == 0) {
#pragma unroll
                for (int q = 0; q < PW / 16; ++q)
                    gstore<uint4>(dp + 16 * q, make_uint4(pw[4 * q], pw[4 * q + 1], pw[4 * q + 2], pw[4 * q + 3]));
            } else {
#pragma unroll
                for (int j = 0; j < PW; ++j)
                    if (j < wc) gstore<uint8_t>(dp + j, (uint8_t)(pw[j >> 2] >> (8 * (j & 3))));
            }
            uint8_t* tp = Wx + cols + r;
#pragma unroll
            for (int t = 0; t < PW; ++t)
                if (t < rp) gstore<uint8_t>(tp + t, (uint8_t)(fw[t >> 2] >> (8 * (t & 3))));
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
            // segment 0: data columns right of the panel; segment 1: transformation
            // columns of the pivots of earlier panels
            for (int seg = 0; seg < 2; ++seg) {
                const int ybase = seg == 0 ? c0 + wc : cols;
                const int ny = seg == 0 ? cols - (c0 + wc) : r;
                for (int ch = 0; ch < ny; ch += VCH) {
                    const int nc = min(VCH, ny - ch);
                    // pivot rows of this chunk, transposed into Vt[column][pivot]
                    for (int i = x; i < rp * (VCH / 16); i += nthr) {
                        const int t = i / (VCH / 16), cb = (i % (VCH / 16)) * 16;
                        if (cb < nc) {
                            const uint8_t* src = e.work + (int64_t)prl[r + t] * e.ldw + ybase + ch + cb;
                            const uint4 v = load16_lim(src, ny - ch - cb);
#pragma unroll
                            for (int bb = 0; bb < 16; ++bb) {
                                const uint32_t wv = bb < 4 ? v.x : bb < 8 ? v.y : bb < 12 ? v.z : v.w;
                                uint32_t byte = (wv >> (8 * (bb & 3))) & 0xffu;
                                if (adj && byte >= 128) byte += adj;
                                Vt[(cb + bb) * FL_ROW + t] = (uint8_t)byte;
                            }
                        }
                    }
                    __syncthreads();
                    // products F * V, reduced mod p, staged as bytes: lane holds row
                    // rb*16 + lane%16 and columns cb*16 + 4*(lane/16) .. +3
                    const int nb = (rows16 >> 4) * (VCH / 16);
                    for (int b = wave; b < nb; b += nwaves) {
                        const int rb = b / (VCH / 16), cb = b % (VCH / 16);
                        const v4i av = *(const v4i*)(Fl + (rb * 16 + (lane & 15)) * FL_ROW + (lane >> 4) * 16);
                        const v4i bv = *(const v4i*)(Vt + (cb * 16 + (lane & 15)) * FL_ROW + (lane >> 4) * 16);
                        const v4i acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(bv, av, v4i{0, 0, 0, 0}, 0, 0, 0);
                        uint32_t word = 0;
#pragma unroll
                        for (int ee = 0; ee < 4; ++ee) word |= mod(acc[ee]) << (8 * ee);
                        *(uint32_t*)(St + (rb * 16 + (lane & 15)) * VCH + cb * 16 + (lane >> 4) * 4) = word;
                    }
                    __syncthreads();
                    // row x: W := (pivot of this panel ? 0 : W) + staged, 16 bytes at a time
                    if (x < rows) {
                        uint8_t* dst = e.work + (int64_t)x * e.ldw + ybase + ch;
                        const bool keep_old = !inpanel[x];
                        for (int cb = 0; cb < nc; cb += 16) {
                            const uint4 st = *(const uint4*)(St + x * VCH + cb);
                            uint4 nv = st;
                            if (keep_old) {
                                const uint4 old = load16_lim(dst + cb, ny - ch - cb);
                                nv = make_uint4(addmod4(old.x, st.x, p), addmod4(old.y, st.y, p),
                                                addmod4(old.z, st.z, p), addmod4(old.w, st.w, p));
                            }
                            const int n = min(16, nc - cb);
                            if (n == 16 && (((uintptr_t)(dst + cb)) & 15) == 0) {
                                gstore<uint4>(dst + cb, nv);
                            } else {
#pragma unroll
                                for (int bb = 0; bb < 16; ++bb) {
                                    const uint32_t wv = bb < 4 ? nv.x : bb < 8 ? nv.y : bb < 12 ? nv.z : nv.w;
                                    if (bb < n) gstore<uint8_t>(dst + cb + bb, (uint8_t)(wv >> (8 * (bb & 3))));
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
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
    // non-pivot rows and columns, ascending: the position of an unselected row
    // (column) is the number of unselected rows (columns) before it, counted a
    // wave-wide ballot at a time
    if (wave == 0) {
        int base = 0;
        for (int r0 = 0; r0 < rows; r0 += 64) {
            const int rr = r0 + lane;
            const bool un = rr < rows && !sel[rr];
            const unsigned long long b = __ballot(un);
            if (un) e.qrow[base + __popcll(b & ((1ull << lane) - 1))] = rr;
            base += __popcll(b);
        }
    }
    if (wave == (nwaves > 1 ? 1 : 0)) {
        // pcl is ascending: column y is a pivot column iff it equals pcl[t] for
        // t = (pivot columns below y); walk it with a per-lane binary search
        int base = 0;
        for (int y0 = 0; y0 < cols; y0 += 64) {
            const int y = y0 + lane;
            int lo = 0, hi = r;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (pcl[mid] < y) lo = mid + 1; else hi = mid;
            }
            const bool np = y < cols && !(lo < r && pcl[lo] == y);
            const unsigned long long b = __ballot(np);
            if (np) e.qcol[base + __popcll(b & ((1ull << lane) - 1))] = y;
            base += __popcll(b);
        }
        for (int y = lane; y < e.qtail; y += 64) e.qcol[base + y] = cols + y;
    }
    __syncthreads();
    for (int t = wave; t < r; t += nwaves) {
        const uint8_t* src = e.work + (int64_t)prl[t] * e.ldw;
        for (int u = lane; u < r; u += 64) gstore<uint8_t>(e.Mo + (int64_t)t * e.ldm + u, gload<uint8_t>(src + cols + u));
        for (int k2 = lane; k2 < cols - r; k2 += 64)
            gstore<uint8_t>(e.Ro + (int64_t)t * e.ldr + k2, gload<uint8_t>(src + gload<int32_t>(e.qcol + k2)));
    }
    for (int s2 = wave; s2 < rows - r; s2 += nwaves) {
        const uint8_t* src = e.work + (int64_t)gload<int32_t>(e.qrow + s2) * e.ldw + cols;
        for (int u = lane; u < r; u += 64) gstore<uint8_t>(e.Ko + (int64_t)s2 * e.ldk + u, gload<uint8_t>(src + u));
    }
}

// ============================================================================ ECH, at most 256 rows, p <= 46
//
// The same elimination as k_ech_panel (columns in order; the pivot of a
// column is the first not-yet-selected row with a non-zero entry; pivot rows
// scaled to -1 and kept reduced against each other; outputs as in EchDesc),
// for blocks of at most 256 rows over GF(p), p <= 46, with the whole working
// matrix W = [H | T] held in LDS (row length LW: the columns of H, padded to
// 16, then the transformation columns, one per pivot).  Eight waves.
//
// Columns go in panels of 32.  A panel's pivots are found by wave 0 alone
// over the first (up to) 64 unselected rows, one row per lane (no row after
// them can be a pivot while one of them is a candidate): a lane holds its
// row's 32 panel entries and its row of the panel transformation F as 16-bit
// pairs, unreduced (an entry receives at most 32 products, each at most
// (p - 1)^2 <= 45^2, so it stays below 2^16).  A pivot step: a ballot picks
// the first candidate with a non-zero entry (the paper's pivot rule), the
// pivot's lane publishes its words in LDS, every lane reduces one of the 64
// published entries, and every lane reads the reduced row back and updates
// its own with one packed 16-bit multiply-add per word; -1/pivot comes from a
// register table (lane v holds -1/v) read across lanes.  The search runs at
// raised wave priority.  The panel's pivot rows are then known as
// combinations G of the original rows, every other row is cleared by them
// with its own entries at the pivot columns as coefficients, and one MFMA
// pass (F = W G per block of 16 rows) applies it all:
//     W[x][y] := (x a pivot of this panel ? 0 : W[x][y]) + sum_t F[x][t] W[pivot row t][y]
// over the later columns and the transformation columns of earlier pivots,
// in units of 16 columns, the B operand read from the pivot rows themselves
// with ds_read_b64_tr_b8.  The next panel's two units go first, split by
// rows over all eight waves (every wave reads its B operand before any of
// them writes: pivot rows are written too); then wave 0 searches the next
// panel while waves 1 to 7 update the remaining units, each unit by one wave
// over every row.  When a column of the search has no candidate while later
// unselected rows exist, the panel goes to the four-wave elimination
// instead: threads 0..255 own rows 0..255, each pivot step takes two
// barriers (each wave posts the ballot of its candidate rows, every thread
// picks the first candidate; the pivot row's thread publishes its words, the
// lanes of its wave reduce the 64 entries, one each, and after the second
// barrier every thread reads them and updates its row).
constexpr int ECHS_MAX_ROWS = 256;
constexpr int ECHS_MAX_P = 46;
constexpr int ECHS_THREADS = 512;
constexpr int ECHS_PW = 32;        // panel width
// LDS layout: the fixed part first (every offset a multiple of 16)
//   pb      96 dwords: [0, 32) published words, [32, 64) reduced, [64] -1/pivot
//           (four-wave elimination), [65] the search's pivot count, [72, 88)
//           two sets of four wave ballots
//   prl, pcl, qrl   256 ints each: pivot rows, pivot columns, non-pivot rows
//   invt    64 dwords: -1/v mod p
//   sel, inpanels   256 bytes, 2 x 256 bytes
//   Gt      32 x 32 bytes: G^T of the panel found by the search
// then F (rows16 x 32 bytes) and W (rows16 x LW bytes).
constexpr int ECHS_OFF_PRL = 384, ECHS_OFF_PCL = 1408, ECHS_OFF_QRL = 2432, ECHS_OFF_INVT = 3456;
constexpr int ECHS_OFF_SEL = 3712, ECHS_OFF_INP = 3968, ECHS_OFF_GT = 4480, ECHS_FIXED = 5504;

__host__ __device__ inline int echs_tc(int cols) { return (cols + 15) & ~15; }
__host__ __device__ inline int echs_lw(int cols, int maxr) { return echs_tc(cols) + ((maxr + 15) & ~15); }
__host__ __device__ inline size_t echs_lds_bytes(int rows, int cols) {
    const int maxr = rows < cols ? rows : cols;
    const size_t rows16 = (size_t)((rows + 15) & ~15);
    return (size_t)ECHS_FIXED + rows16 * ECHS_PW + rows16 * (size_t)echs_lw(cols, maxr);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
// two 16-bit multiply-adds: (a.lo * b.lo + c.lo, a.hi * b.hi + c.hi), mod 2^16
__device__ __forceinline__ uint32_t pkmad16(uint32_t a, uint32_t b, uint32_t c) {
    const u16x2 r = __builtin_bit_cast(u16x2, a) * __builtin_bit_cast(u16x2, b) + __builtin_bit_cast(u16x2, c);
    return __builtin_bit_cast(uint32_t, r);
}

// acc[w] += f2 * v[w] in 16-bit halves, w < NW
template <int NW>
__device__ __forceinline__ void pkmad_words(uint32_t* acc, const uint32_t* v, uint32_t f2) {
#pragma unroll
    for (int w = 0; w < NW; ++w) acc[w] = pkmad16(f2, v[w], acc[w]);
}

// Orders the LDS accesses of one wave around it (the wave's LDS operations
// complete in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v mod p for 0 <= v < 2^17, given inv17 = fl(fl(1/p) (1 + 2^-18)) (fl(1/p)
// within an ulp or two): fl(v inv17) = (v / p)(1 + e) with 0 < e < 2^-17, so it
// is at least v / p and below floor(v / p) + 1 (v e < 1 <= p - v mod p), and
// its integer part is floor(v / p) exactly.  For every p <= 251 and v < 2^17
// this is checked exhaustively on the host in float32 arithmetic.
__device__ __forceinline__ uint32_t mod17(uint32_t v, float inv17, uint32_t p) {
    const int q = (int)((float)v * inv17);
    return (uint32_t)(__mul24(q, -(int)p) + (int)v);
}

// byte u (when 0 <= u < 4) of w, a residue, less one mod p
__device__ __forceinline__ uint32_t echs_dec_byte(uint32_t w, int u, uint32_t p) {
    if (u < 0 || u >= 4) return w;
    const uint32_t sh = 8u * (uint32_t)u, b = (w >> sh) & 0xffu;
    return (w & ~(0xffu << sh)) | ((b ? b - 1u : p - 1u) << sh);
}

// 32 panel entries of a row (bytes at p, `wc` of them valid) as 16 words of
// 16-bit pairs: column k in half (k & 1) of word k / 2
__device__ __forceinline__ void echs_unpack_panel(const uint8_t* p, bool ok, int wc, uint32_t* D) {
    uint4 a = make_uint4(0, 0, 0, 0), b = make_uint4(0, 0, 0, 0);
    if (ok) {
        a = *(const uint4*)p;
        b = *(const uint4*)(p + 16);
    }
    const uint32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint32_t lo = __builtin_amdgcn_perm(0u, d[i], 0x0c010c00u);
        uint32_t hi = __builtin_amdgcn_perm(0u, d[i], 0x0c030c02u);
        if (wc < ECHS_PW) {   // columns past the block hold other data: clear them
            if (4 * i >= wc) lo &= 0u; else if (4 * i + 1 >= wc) lo &= 0xffffu;
            if (4 * i + 2 >= wc) hi &= 0u; else if (4 * i + 3 >= wc) hi &= 0xffffu;
        }
        D[2 * i] = lo;
        D[2 * i + 1] = hi;
    }
}

template <class Src>
__global__ void __launch_bounds__(ECHS_THREADS) k_ech_lds(Src src) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int NW = ECHS_THREADS / 64;
    const EchDesc e = src.get(blockIdx.x);
    const int rows = e.rows, cols = e.cols;
    const int maxr = rows < cols ? rows : cols;
    const int TC = echs_tc(cols), LW = echs_lw(cols, maxr);
    const int rows16 = (rows + 15) & ~15, nrb = rows16 >> 4;
    const uint32_t p = (uint32_t)e.p;
    const float inv = 1.0f / (float)p;
    const float inv17 = inv * (1.0f + 0x1p-18f);
    // the wave index is uniform: reading it through the first lane lets the
    // compiler keep what depends on it in scalar registers
    const int x = threadIdx.x, lane = x & 63, wave = __builtin_amdgcn_readfirstlane(x >> 6);

    uint32_t* const pb = (uint32_t*)smem;
    unsigned long long* const mskb = (unsigned long long*)(pb + 72);
    int* const prl = (int*)(smem + ECHS_OFF_PRL);
    int* const pcl = (int*)(smem + ECHS_OFF_PCL);
    int* const qrl = (int*)(smem + ECHS_OFF_QRL);
    uint32_t* const invt = (uint32_t*)(smem + ECHS_OFF_INVT);
    uint8_t* const sel = smem + ECHS_OFF_SEL;
    uint8_t* const inpanels = smem + ECHS_OFF_INP;
    uint8_t* const Gt = smem + ECHS_OFF_GT;      // Gt[s][t]: coefficient of original pivot row s in the panel's pivot row t
    uint8_t* const Fl = smem + ECHS_FIXED;       // [rows16][32]
    uint8_t* const W = Fl + rows16 * ECHS_PW;    // [rows16][LW]

    // -1/v mod p for v = lane (0 for v = 0 and v >= p): v^(p - 2) = 1/v (Fermat)
    uint32_t ninv = 0;
    {
        uint32_t b = (uint32_t)lane < p ? (uint32_t)lane : 0u, a = 1u;
        for (uint32_t ex = p - 2; ex; ex >>= 1) {
            if (ex & 1u) a = mod22(a * b, inv, p);
            b = mod22(b * b, inv, p);
        }
        ninv = (lane > 0 && (uint32_t)lane < p) ? p - a : 0u;
    }
    if (x < 64) invt[x] = ninv;
    for (int i = x; i < 256; i += ECHS_THREADS) { sel[i] = 0; inpanels[i] = 0; inpanels[256 + i] = 0; }
    // W = [H | 0], rows beyond `rows` zero.  Thread x covers 16-byte chunks
    // x, x + 512, ...; the loads of 8 chunks are in flight together.
    {
        const int cpr = LW >> 4;                     // chunks per row
        const int nch = rows16 * cpr;
        const bool hal = ((((uintptr_t)e.H) | (uintptr_t)e.ldh) & 15) == 0;
        for (int c0 = x; c0 < nch; c0 += 8 * ECHS_THREADS) {
            uint4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * ECHS_THREADS;
                v[u] = make_uint4(0, 0, 0, 0);
                if (c < nch) {
                    const int rr = c / cpr, y = (c - rr * cpr) * 16;
                    if (rr < rows && y < cols) {
                        const uint8_t* sp = e.H + (int64_t)rr * e.ldh + y;
                        v[u] = (hal && y + 16 <= cols) ? gload<uint4>(sp) : load16_lim(sp, cols - y);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * ECHS_THREADS;
                if (c < nch) *(uint4*)(W + (size_t)c * 16) = v[u];
            }
        }
    }
    __syncthreads();

    int r = 0;
    bool my_sel = x >= rows;     // thread x < 256 owns row x in the four-wave elimination
    int* const act = qrl;        // the search's candidate rows (scratch until the outputs)
    // Panel c0's search (wave 0) runs in the iteration of the panel before
    // it, beside that panel's trailing update; the iteration at c0 = -32 only
    // searches panel 0.  The two inpanel arrays alternate by panel, so the
    // search can mark the next panel's pivots while the update still reads
    // the current panel's.
    for (int c0 = -ECHS_PW; c0 < cols && r < maxr; c0 += ECHS_PW) {
        const int pi = (c0 + ECHS_PW) / ECHS_PW;
        uint8_t* const inpanel = inpanels + 256 * (pi & 1);          // the current panel's pivots
        uint8_t* const inpanel_nx = inpanels + 256 * ((pi + 1) & 1); // the next panel's
        const int nc0 = c0 + ECHS_PW;
        int rp = 0, fast_rp = -1;
        if (c0 >= 0) {
            const int wc = min(ECHS_PW, cols - c0);
            fast_rp = __builtin_amdgcn_readfirstlane((int)pb[65]);
            my_sel = x >= rows || sel[x];
            if (fast_rp >= 0) {
                rp = fast_rp;
                if (rp > 0) {
                    // F = Wc G by MFMA (K = 32, one row block of 16 rows per step):
                    // Wc[x][t] = W[x][pivot column t] for a row that is not a pivot of
                    // this panel, the unit vector e_t for the panel's pivot t (its F row
                    // is G's row t); entries t >= rp are zero.  The lanes of a quarter
                    // hold k = kq .. kq + 7; the output lane holds F[row][4 (lane / 16) + j]
                    // and F[row][16 + 4 (lane / 16) + j].
                    const int kq = (lane >> 4) * 8;
                    const bool contig = pcl[r + rp - 1] == c0 + rp - 1;   // pivot columns c0 .. c0 + rp - 1
                    int pcol[8];
                    uint64_t kmask = 0;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const bool in = kq + j < rp;
                        pcol[j] = in ? pcl[r + kq + j] : -1;
                        if (in) kmask |= 0xffull << (8 * j);
                    }
                    const long bv0 = *(const long*)(Gt + (lane & 15) * ECHS_PW + kq);
                    const long bv1 = *(const long*)(Gt + (16 + (lane & 15)) * ECHS_PW + kq);
                    for (int rb = wave; rb < nrb; rb += NW) {
                        const int row = rb * 16 + (lane & 15);
                        const int ip = row < rows ? (int)inpanel[row] : 0;
                        uint64_t av = 0;
                        if (row < rows) {
                            const uint8_t* wr = W + (size_t)row * LW;
                            if (ip) {
                                const int u = ip - 1 - kq;
                                av = (u >= 0 && u < 8) ? 1ull << (8 * u) : 0ull;
                            } else if (contig) {
                                av = *(const uint64_t*)(wr + c0 + kq) & kmask;
                            } else {
#pragma unroll
                                for (int j = 0; j < 8; ++j)
                                    if (pcol[j] >= 0) av |= (uint64_t)wr[pcol[j]] << (8 * j);
                            }
                        }
                        const v4i f0 = __builtin_amdgcn_mfma_i32_16x16x32_i8(bv0, (long)av, v4i{0, 0, 0, 0}, 0, 0, 0);
                        const v4i f1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(bv1, (long)av, v4i{0, 0, 0, 0}, 0, 0, 0);
                        uint32_t w0 = 0, w1 = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            w0 |= mod17((uint32_t)f0[j], inv17, p) << (8 * j);
                            w1 |= mod17((uint32_t)f1[j], inv17, p) << (8 * j);
                        }
                        const int s0 = (lane >> 4) * 4;
                        if (row < rows) {
                            uint8_t* wt = W + (size_t)row * LW + TC + r;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                if (s0 + j < rp) wt[s0 + j] = (uint8_t)(w0 >> (8 * j));
                                if (16 + s0 + j < rp) wt[16 + s0 + j] = (uint8_t)(w1 >> (8 * j));
                            }
                        }
                        // the update adds F W[pivot rows] to every row: a pivot row's F is
                        // G's row less its own unit vector
                        if (ip) {
                            w0 = echs_dec_byte(w0, ip - 1 - s0, p);
                            w1 = echs_dec_byte(w1, ip - 1 - 16 - s0, p);
                        }
                        *(uint32_t*)(Fl + row * ECHS_PW + s0) = w0;
                        *(uint32_t*)(Fl + row * ECHS_PW + 16 + s0) = w1;
                    }
                }
            } else {
                // Four-wave elimination of the panel (threads 0..255; the other
                // waves take part in the barriers only)
                const bool ok = x < rows;
                uint32_t D[16], F[16];
                uint32_t scale = 1;
                int pidx = -1;
                echs_unpack_panel(W + (size_t)x * LW + c0, ok, wc, D);
#pragma unroll
                for (int w = 0; w < 16; ++w) F[w] = 0;
                // Column k of the panel (k static, so every register index is).  Every
                // decision below is taken from LDS values all threads read alike, so
                // rp stays uniform.
                static_for<0, ECHS_PW>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    if (k >= wc || r + rp >= maxr) return;
                    constexpr int wk = k >> 1, hk = 16 * (k & 1);
                    const uint32_t red = mod22((D[wk] >> hk) & 0xffffu, inv, p);
                    const unsigned long long bm = __ballot(!my_sel && red != 0u);
                    // by column parity: a column without a pivot has no second barrier
                    unsigned long long* msk = mskb + 4 * (k & 1);
                    if (lane == 0 && wave < 4) msk[wave] = bm;
                    __syncthreads();
                    const unsigned long long m0w = msk[0], m1w = msk[1], m2w = msk[2], m3w = msk[3];
                    const int Q = m0w ? 0 : m1w ? 1 : m2w ? 2 : m3w ? 3 : -1;
                    if (Q < 0) return;    // no candidate row: not a pivot column
                    const unsigned long long mq = Q == 0 ? m0w : Q == 1 ? m1w : Q == 2 ? m2w : m3w;
                    const int prow = 64 * Q + (__ffsll((long long)mq) - 1);   // first candidate row
                    const bool me = x == prow;
                    if (me) {
                        // publish the row's unreduced words; its own transformation
                        // entry (index rp) is 1; and -1 / pivot
                        const uint32_t sv = invt[red];
                        const uint32_t one = 1u << (16 * (rp & 1));
#pragma unroll
                        for (int w = 0; w < 16; w += 4) {
                            *(uint4*)(pb + w) = make_uint4(D[w], D[w + 1], D[w + 2], D[w + 3]);
                            *(uint4*)(pb + 16 + w) = make_uint4(
                                F[w] + (w == (rp >> 1) ? one : 0u), F[w + 1] + (w + 1 == (rp >> 1) ? one : 0u),
                                F[w + 2] + (w + 2 == (rp >> 1) ? one : 0u), F[w + 3] + (w + 3 == (rp >> 1) ? one : 0u));
                        }
                        pb[64] = sv;
                    }
                    if (wave == Q) {
                        // the pivot's wave reduces the 64 published entries, one per lane
                        wave_sync();
                        ((uint16_t*)(pb + 32))[lane] = (uint16_t)mod22(((const uint16_t*)pb)[lane], inv, p);
                    }
                    __syncthreads();
                    uint32_t pv[32];
#pragma unroll
                    for (int w = 0; w < 32; w += 4) {
                        const uint4 t4 = *(const uint4*)(pb + 32 + w);
                        pv[w] = t4.x; pv[w + 1] = t4.y; pv[w + 2] = t4.z; pv[w + 3] = t4.w;
                    }
                    const uint32_t sv = pb[64];
                    const uint32_t f = me ? 0u : mod22(__umul24(red, sv), inv, p);
                    const uint32_t f2 = f * 0x10001u;
                    // the reduced pivot row is zero in the panel's earlier columns and
                    // in transformation entries past rp <= k
#pragma unroll
                    for (int w = wk; w < 16; ++w) D[w] = pkmad16(f2, pv[w], D[w]);
#pragma unroll
                    for (int w = 0; w <= wk; ++w) F[w] = pkmad16(f2, pv[16 + w], F[w]);
                    if (me) {
                        my_sel = true;
                        scale = sv;
                        pidx = rp;
                        prl[r + rp] = prow;
                        pcl[r + rp] = c0 + k;
                        sel[prow] = 1;
                        inpanel[prow] = 1;
                    }
                    ++rp;
                });
                rp = __builtin_amdgcn_readfirstlane(rp);
                // reduce, give the pivot row its own transformation entry 1 and scale
                // it to pivot -1, then write the panel, F (for the MFMA) and the new
                // transformation columns (F itself) back to LDS
                if (ok) {
                    uint32_t pk[8], fk[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        uint32_t v[4], g[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int col = 4 * i + j;
                            const uint32_t wd = D[col >> 1], fw = F[col >> 1];
                            const uint32_t dv = (col & 1) ? (wd >> 16) : (wd & 0xffffu);
                            uint32_t fv = (col & 1) ? (fw >> 16) : (fw & 0xffffu);
                            if (col == pidx) fv += 1;
                            v[j] = mod22(__umul24(dv, scale), inv, p);
                            g[j] = mod22(__umul24(fv, scale), inv, p);
                        }
                        pk[i] = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
                        fk[i] = g[0] | (g[1] << 8) | (g[2] << 16) | (g[3] << 24);
                    }
                    uint8_t* wr = W + (size_t)x * LW;
                    if (wc == ECHS_PW) {
                        *(uint4*)(wr + c0) = make_uint4(pk[0], pk[1], pk[2], pk[3]);
                        *(uint4*)(wr + c0 + 16) = make_uint4(pk[4], pk[5], pk[6], pk[7]);
                    } else {
#pragma unroll
                        for (int j = 0; j < ECHS_PW; ++j)
                            if (j < wc) wr[c0 + j] = (uint8_t)(pk[j >> 2] >> (8 * (j & 3)));
                    }
#pragma unroll
                    for (int t = 0; t < ECHS_PW; ++t)
                        if (t < rp) wr[TC + r + t] = (uint8_t)(fk[t >> 2] >> (8 * (t & 3)));
                    if (pidx >= 0) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) fk[i] = echs_dec_byte(fk[i], pidx - 4 * i, p);
                    }
                    *(uint4*)(Fl + x * ECHS_PW) = make_uint4(fk[0], fk[1], fk[2], fk[3]);
                    *(uint4*)(Fl + x * ECHS_PW + 16) = make_uint4(fk[4], fk[5], fk[6], fk[7]);
                } else if (x < rows16) {   // rows past `rows` (padding of the MFMA tiles)
                    *(uint4*)(Fl + x * ECHS_PW) = make_uint4(0, 0, 0, 0);
                    *(uint4*)(Fl + x * ECHS_PW + 16) = make_uint4(0, 0, 0, 0);
                }
            }
            __syncthreads();
        }
        const bool next = nc0 < cols && r + rp < maxr;
        if (rp > 0) {
            // Trailing update in units of 16 columns: units [0, n0u) the data
            // columns from ybeg on (from the next panel when the four-wave
            // elimination has written this one), units [n0u, nu) the
            // transformation columns of earlier pivots.  Lane l's B operand is
            // 8 bytes of pivot row kk at column y0 + 8 (l & 1); the MFMA gives
            // lane l the row rb * 16 + (l & 15) at columns 4 (l / 16) .. + 3.
            const int ybeg = fast_rp >= 0 ? c0 : nc0;
            const int n0u = ybeg < cols ? (cols - ybeg + 15) >> 4 : 0;
            const int nu = n0u + ((r + 15) >> 4);
            const int kk = (lane >> 4) * 8 + ((lane & 15) >> 1);
            const int po = (kk < rp ? prl[r + kk] : prl[r]) * LW + ((lane & 1) << 3);
            const int cc = (lane >> 4) * 4;
            const auto ucol = [&](int u, int& y0, int& nc) {
                if (u < n0u) {
                    y0 = ybeg + 16 * u;
                    nc = min(16, cols - y0);
                } else {
                    y0 = TC + 16 * (u - n0u);
                    nc = min(16, TC + r - y0);
                }
            };
            const auto bfrag = [&](int y0) { return __builtin_bit_cast(long, lds_read_tr8(W + po + y0)); };
            // W[row][y0 + cc + j] += sum_t F[row][t] W[pivot row t][y0 + cc + j]: the
            // old bytes enter as the MFMA's accumulator; bytes past the unit's nc
            // columns are kept
            const auto apply = [&](int y0, int nc, long b, int rb) {
                const int row = rb * 16 + (lane & 15);
                const long av = *(const long*)(Fl + row * ECHS_PW + (lane >> 4) * 8);
                uint32_t* wp = (uint32_t*)(W + (size_t)row * LW + y0 + cc);
                const uint32_t old = *wp;
                const v4i c = {(int)(old & 0xffu), (int)((old >> 8) & 0xffu), (int)((old >> 16) & 0xffu),
                               (int)(old >> 24)};
                const v4i acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(b, av, c, 0, 0, 0);
                if (row < rows && cc < nc) {
                    uint32_t out = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) out |= mod17((uint32_t)acc[j], inv17, p) << (8 * j);
                    const uint32_t keep = nc - cc >= 4 ? 0u : 0xffffffffu << (8 * (nc - cc));
                    *wp = (out & ~keep) | (old & keep);
                }
            };
            const auto unit = [&](int u) {      // one unit, every row, by one wave
                int y0, nc;
                ucol(u, y0, nc);
                const long b = bfrag(y0);
#pragma unroll 2
                for (int rb = 0; rb < nrb; ++rb) apply(y0, nc, b, rb);
            };
            if (next) {
                // the next panel's columns (units qa and qa + 1) first, by rows over
                // all waves; every wave reads its B operands before any wave writes
                const int qa = (nc0 - ybeg) >> 4;
                const bool two = qa + 1 < n0u;
                int ya, na, yb = 0, nb = 0;
                ucol(qa, ya, na);
                if (two) ucol(qa + 1, yb, nb);
                const long ba = bfrag(ya);
                const long bb = two ? bfrag(yb) : 0;
                __syncthreads();
                for (int rb = wave; rb < nrb; rb += NW) {
                    apply(ya, na, ba, rb);
                    if (two) apply(yb, nb, bb, rb);
                }
                __syncthreads();
                // the other units, one wave each, beside the search
                const int skip = two ? 2 : 1;
                for (int i = wave - 1; wave > 0 && i < nu - skip; i += NW - 1) unit(i < qa ? i : i + skip);
            } else {
                for (int u = wave; u < nu; u += NW) unit(u);
            }
        }
        if (next && wave == 0) {
            // the next panel's columns are final: search it
            __builtin_amdgcn_s_setprio(3);
            const int c0 = nc0, r_nx = r + rp;
            const int r = r_nx;
            uint8_t* const inpanel = inpanel_nx;
            const int wc = __builtin_amdgcn_readfirstlane(min(ECHS_PW, cols - c0));
            int total = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 64 * q + lane;
                const bool un = row < rows && !sel[row];
                const unsigned long long bq = __ballot(un);
                const int pos = total + __popcll(bq & ((1ull << lane) - 1));
                if (un && pos < 64) act[pos] = row;
                total += __popcll(bq);
            }
            wave_sync();
            const int arow = lane < total ? act[lane] : -1;
            const bool spill = total > 64;
            uint32_t D[16], F[16];
            echs_unpack_panel(W + (size_t)(arow >= 0 ? arow : 0) * LW + c0, arow >= 0, wc, D);
#pragma unroll
            for (int w = 0; w < 16; ++w) F[w] = 0;
            // selected lanes (a lane without a candidate row counts as one), as a mask
            unsigned long long selm = __ballot(arow < 0);
            bool nocand = false;   // a column of the block where no candidate is non-zero
            uint32_t scale = 1;
            int pidx = -1, rpa = 0;
            // Steps in groups of 8; a group runs while the panel has columns left
            // and some candidate is unselected.  Within a group every step runs,
            // branch-free: past the panel's columns (zeroed by the unpacking) no
            // lane is a candidate and the step changes nothing.
            static_for<0, ECHS_PW / 8>([&](auto gc) {
                constexpr int g = decltype(gc)::value;
                if (__builtin_amdgcn_readfirstlane((int)(8 * g >= wc || selm == ~0ull))) return;
                static_for<8 * g, 8 * g + 8>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int wk = k >> 1, hk = 16 * (k & 1);
                    const uint32_t red = mod17((D[wk] >> hk) & 0xffffu, inv17, p);
                    const unsigned long long bm = __ballot(red != 0u) & ~selm;
                    nocand = nocand | ((bm == 0) & (k < wc));
                    const int P = bm ? __ffsll((long long)bm) - 1 : 0;
                    const bool me = bm != 0 && lane == P;
                    const uint32_t sv = __builtin_amdgcn_readlane(ninv, __builtin_amdgcn_readlane(red, P));
                    if (me) {
#pragma unroll
                        for (int w = 0; w < 16; w += 4) {
                            *(uint4*)(pb + w) = make_uint4(D[w], D[w + 1], D[w + 2], D[w + 3]);
                            *(uint4*)(pb + 16 + w) = make_uint4(F[w], F[w + 1], F[w + 2], F[w + 3]);
                        }
                        prl[r + rpa] = arow;
                        pcl[r + rpa] = c0 + k;
                    }
                    wave_sync();
                    // lane j reduces published entry j; the pivot's own transformation
                    // entry (index 32 + rpa, zero so far) becomes 1
                    ((uint16_t*)(pb + 32))[lane] =
                        (uint16_t)(mod17(((const uint16_t*)pb)[lane], inv17, p) + (lane == 32 + rpa ? 1u : 0u));
                    wave_sync();
                    uint32_t pv[32];
#pragma unroll
                    for (int w = 0; w < 32; w += 4) {
                        const uint4 t4 = *(const uint4*)(pb + 32 + w);
                        pv[w] = t4.x; pv[w + 1] = t4.y; pv[w + 2] = t4.z; pv[w + 3] = t4.w;
                    }
                    const uint32_t f = mod17(__umul24(red, sv), inv17, p);
                    const uint32_t f2 = (bm != 0 && !me) ? f * 0x10001u : 0u;
#pragma unroll
                    for (int w = wk; w < 16; ++w) D[w] = pkmad16(f2, pv[w], D[w]);
#pragma unroll
                    for (int w = 0; w <= wk; ++w) F[w] = pkmad16(f2, pv[16 + w], F[w]);
                    scale = me ? sv : scale;
                    pidx = me ? rpa : pidx;
                    selm |= bm & (~bm + 1ull);
                    rpa = __builtin_amdgcn_readfirstlane(rpa + (bm != 0 ? 1 : 0));
                    wave_sync();
                });
            });
            __builtin_amdgcn_s_setprio(0);
            // no candidate in a column of the block while later unselected rows
            // exist: the four-wave elimination takes the panel
            const bool fb = spill && nocand;
            if (!fb && pidx >= 0) {
                // G row pidx = scale (F + e_pidx), reduced, as 16 words of 16-bit pairs
#pragma unroll
                for (int w = 0; w < 16; ++w) {
                    const uint32_t fw = F[w];
                    uint32_t lo = fw & 0xffffu, hi = fw >> 16;
                    if (2 * w == pidx) lo += 1;
                    if (2 * w + 1 == pidx) hi += 1;
                    F[w] = mod22(__umul24(lo, scale), inv, p) | (mod22(__umul24(hi, scale), inv, p) << 16);   // lo, hi < 2^16
                }
#pragma unroll
                for (int w = 0; w < 16; ++w) {
                    Gt[(2 * w) * ECHS_PW + pidx] = (uint8_t)F[w];
                    Gt[(2 * w + 1) * ECHS_PW + pidx] = (uint8_t)(F[w] >> 16);
                }
                sel[arow] = 1;
                inpanel[arow] = (uint8_t)(pidx + 1);
            }
            if (lane == 0) pb[65] = fb ? 0xffffffffu : (uint32_t)rpa;
        }
        __syncthreads();
        for (int t = x; t < rp; t += ECHS_THREADS) inpanel[prl[r + t]] = 0;
        r += rp;
    }
    // ---- outputs
    const int nq = cols - r;
    int* const qcl = (int*)Fl;                       // the non-pivot columns, when they fit
    const bool qin = nq <= rows16 * (ECHS_PW / 4);
    if (x == 0) *e.rcount = r;
    for (int t = x; t < r; t += ECHS_THREADS) {
        e.prow[t] = prl[t];
        e.pcol[t] = pcl[t];
    }
    if (wave == 0) {
        int base = 0;
        for (int r0 = 0; r0 < rows; r0 += 64) {
            const int rr = r0 + lane;
            const bool un = rr < rows && !sel[rr];
            const unsigned long long bq = __ballot(un);
            if (un) {
                const int pos = base + __popcll(bq & ((1ull << lane) - 1));
                e.qrow[pos] = rr;
                qrl[pos] = rr;
            }
            base += __popcll(bq);
        }
    }
    // the non-pivot columns: column y, not a pivot, goes to position y less the
    // number of pivot columns before it (pcl is increasing)
    for (int y = x; y < cols; y += ECHS_THREADS) {
        int lo = 0, hi = r;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pcl[mid] < y) lo = mid + 1; else hi = mid;
        }
        if (!(lo < r && pcl[lo] == y)) {
            e.qcol[y - lo] = y;
            if (qin) qcl[y - lo] = y;
        }
    }
    for (int y = x; y < e.qtail; y += ECHS_THREADS) e.qcol[nq + y] = cols + y;
    __syncthreads();
    // M (rows of the pivots) and K (non-pivot rows) at the transformation
    // columns, 16 bytes per thread; R (pivot rows at the non-pivot columns),
    // 4 bytes per thread
    const int mch = (r + 15) >> 4;
    const bool mal = ((((uintptr_t)e.Mo) | (uintptr_t)e.ldm) & 15) == 0;
    const bool kal = ((((uintptr_t)e.Ko) | (uintptr_t)e.ldk) & 15) == 0;
    for (int i = x; i < rows * mch; i += ECHS_THREADS) {
        const int t = i / mch, c = i - t * mch;
        const bool piv = t < r;
        const int src_row = piv ? prl[t] : qrl[t - r];
        uint8_t* dst = piv ? e.Mo + (int64_t)t * e.ldm : e.Ko + (int64_t)(t - r) * e.ldk;
        const uint4 v = *(const uint4*)(W + (size_t)src_row * LW + TC + 16 * c);
        const int nb = min(16, r - 16 * c);
        if (nb == 16 && (piv ? mal : kal)) {
            gstore<uint4>(dst + 16 * c, v);
        } else {
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
            for (int j = 0; j < nb; ++j) gstore<uint8_t>(dst + 16 * c + j, (uint8_t)(wv[j >> 2] >> (8 * (j & 3))));
        }
    }
    const int rch = (nq + 3) >> 2;
    const bool ral = ((((uintptr_t)e.Ro) | (uintptr_t)e.ldr) & 3) == 0;
    for (int i = x; i < r * rch; i += ECHS_THREADS) {
        const int t = i / rch, k2 = 4 * (i - t * rch);
        const uint8_t* wr = W + (size_t)prl[t] * LW;
        const int nb = min(4, nq - k2);
        uint32_t v = 0;
        for (int j = 0; j < nb; ++j) {
            const int qc = qin ? qcl[k2 + j] : gload<int32_t>(e.qcol + k2 + j);
            v |= (uint32_t)wr[qc] << (8 * j);
        }
        uint8_t* dst = e.Ro + (int64_t)t * e.ldr + k2;
        if (nb == 4 && ral) {
            gstore<uint32_t>(dst, v);
        } else {
            for (int j = 0; j < nb; ++j) gstore<uint8_t>(dst + j, (uint8_t)(v >> (8 * j)));
        }
    }
}

// ============================================================================ small jobs

constexpr int SMALL_THREADS = 256;
constexpr int SMALL_ARG_CAP = 48;      // descriptors passed by value (at most 48 x 80 bytes)

// grid: (x blocks striding over elements, y = descriptor)
// grid: (x blocks striding over rows, y = descriptor); threads stride over columns
template <class Src>
__global__ void __launch_bounds__(SMALL_THREADS) k_gather(Src src) {
    const GatherDesc g = src.get(blockIdx.y);
    constexpr int U = 8;   // elements per thread in flight: the map loads, then the data loads, then the stores
    // rows copied without a column map move as 16-byte chunks
    const bool vec = !g.dcol && !g.neg_p && !g.scol && ((((uintptr_t)g.dst) | (uintptr_t)g.ldd) & 15) == 0 &&
                     ((((uintptr_t)g.src) | (uintptr_t)g.lds) & 3) == 0;
    // a column map onto 16-byte aligned destination rows: by chunks (below)
    const bool runs = !g.dcol && !g.neg_p && g.scol && ((((uintptr_t)g.dst) | (uintptr_t)g.ldd) & 15) == 0 &&
                      ((((uintptr_t)g.src) | (uintptr_t)g.lds) & 3) == 0;
    const bool sal = (((uintptr_t)g.scol) & 15) == 0;
    for (int x = blockIdx.x; x < g.rows; x += gridDim.x) {
        const int64_t sr = g.srow ? gload<int32_t>(g.srow + x) : x;
        const int64_t dr = g.drow ? gload<int32_t>(g.drow + x) : x;
        const uint8_t* src = g.src + sr * g.lds;
        uint8_t* dst = g.dst + dr * g.ldd;
        if (vec) {
            constexpr int V = 4;   // chunks per thread in flight
            for (int c0 = threadIdx.x * 16; c0 < g.cols; c0 += SMALL_THREADS * 16 * V) {
                uint4 v[V];
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    const int c = c0 + u * SMALL_THREADS * 16;
                    v[u] = make_uint4(0, 0, 0, 0);
                    if (c + 16 <= g.cols) {
                        const uint32_t* q = (const uint32_t*)(src + c);
                        v[u] = make_uint4(gload<uint32_t>(q), gload<uint32_t>(q + 1), gload<uint32_t>(q + 2),
                                          gload<uint32_t>(q + 3));
                    }
                }
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    const int c = c0 + u * SMALL_THREADS * 16;
                    if (c >= g.cols) break;
                    if (c + 16 <= g.cols) {
                        gstore<uint4>(dst + c, v[u]);
                    } else {
                        for (int i = c; i < g.cols; ++i) gstore<uint8_t>(dst + i, gload<uint8_t>(src + i));
                    }
                }
            }
            continue;
        }
        if (runs) {
            // 16-byte chunks of the destination row: when the chunk's 16 source
            // columns are consecutive (the column maps of the final assembly are
            // long ascending runs), one realigned 16-byte load
            for (int y = threadIdx.x * 16; y < g.cols; y += SMALL_THREADS * 16) {
                if (y + 16 <= g.cols) {
                    int32_t ix[16];
                    if (sal) {     // the 16 column numbers as four 16-byte loads
#pragma unroll
                        for (int i = 0; i < 16; i += 4) {
                            const uint4 q = gload<uint4>(g.scol + y + i);
                            ix[i] = (int32_t)q.x; ix[i + 1] = (int32_t)q.y; ix[i + 2] = (int32_t)q.z; ix[i + 3] = (int32_t)q.w;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 16; ++i) ix[i] = gload<int32_t>(g.scol + y + i);
                    }
                    // the realigned load reads the dwords around the 16 bytes: up
                    // to 3 bytes past them, which must stay inside the source row
                    bool run = (int64_t)ix[0] + 20 <= g.lds;
#pragma unroll
                    for (int i = 1; i < 16; ++i) run = run && ix[i] == ix[0] + i;
                    uint4 v;
                    if (run) {
                        v = load16_any(src + ix[0]);
                    } else {
                        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                        for (int i = 0; i < 16; ++i) w[i >> 2] |= (uint32_t)gload<uint8_t>(src + ix[i]) << (8 * (i & 3));
                        v = make_uint4(w[0], w[1], w[2], w[3]);
                    }
                    gstore<uint4>(dst + y, v);
                } else {
                    for (int i = y; i < g.cols; ++i) gstore<uint8_t>(dst + i, gload<uint8_t>(src + gload<int32_t>(g.scol + i)));
                }
            }
            continue;
        }
        for (int y0 = threadIdx.x; y0 < g.cols; y0 += SMALL_THREADS * U) {
            int64_t sc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * SMALL_THREADS;
                sc[u] = y < g.cols ? (g.scol ? (int64_t)gload<int32_t>(g.scol + y) : (int64_t)y) : -1;
            }
            uint32_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = sc[u] >= 0 ? (uint32_t)gload<uint8_t>(src + sc[u]) : 0u;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int y = y0 + u * SMALL_THREADS;
                if (y >= g.cols) break;
                uint32_t w = v[u];
                if (g.neg_p) w = (uint32_t)((g.neg_p - (int)w) % g.neg_p);
                const int64_t dc = g.dcol ? gload<int32_t>(g.dcol + y) : y;
                gstore<uint8_t>(dst + dc, (uint8_t)w);
            }
        }
    }
}

template <class Src>
__global__ void __launch_bounds__(SMALL_THREADS) k_fill(Src src) {
    const FillDesc f = src.get(blockIdx.y);
    if (f.dcol) {
        for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < f.rows; t += gridDim.x * SMALL_THREADS)
            f.dst[(int64_t)t * f.ldd + f.dcol[t]] = (uint8_t)f.diag_value;
        return;
    }
    for (int x = blockIdx.x; x < f.rows; x += gridDim.x)
        for (int y = threadIdx.x; y < f.cols; y += SMALL_THREADS)
            gstore<uint8_t>(f.dst + (int64_t)x * f.ldd + y,
                            (uint8_t)((x == y && f.diag_value >= 0) ? f.diag_value : f.value));
}

template <class Src>
__global__ void __launch_bounds__(SMALL_THREADS) k_lists(Src src) {
    const ListDesc l = src.get(blockIdx.y);
    for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < l.npick; t += gridDim.x * SMALL_THREADS) {
        const int u = l.pick ? l.pick[t] : t;
        l.append[t] = l.add + (l.map ? l.map[u] : u);
    }
    for (int s = blockIdx.x * SMALL_THREADS + threadIdx.x; s < l.nkeep; s += gridDim.x * SMALL_THREADS) {
        const int u = l.keep ? l.keep[s] : s;
        l.keep_out[s] = l.map ? l.map[u] : u;
    }
}

// rank sort of distinct values: out[rank(t)] = add + (mode ? t : vals[t])
template <class Src>
__global__ void __launch_bounds__(SMALL_THREADS) k_sort(Src src) {
    const SortDesc s = src.get(blockIdx.y);
    for (int t = blockIdx.x * SMALL_THREADS + threadIdx.x; t < s.n; t += gridDim.x * SMALL_THREADS) {
        int v = s.vals[t], rank = 0;
        for (int u = 0; u < s.n; ++u) rank += s.vals[u] < v;
        s.out[rank] = s.add + (s.mode ? t : v);
    }
}

__global__ void __launch_bounds__(SMALL_THREADS)
k_range(const uint8_t* __restrict__ A, int64_t m, int64_t n, int64_t lda, int p, unsigned long long* bad) {
    unsigned long long cnt = 0;
    for (int64_t x = blockIdx.x; x < m; x += gridDim.x)
        for (int64_t y = threadIdx.x; y < n; y += SMALL_THREADS) cnt += gload<uint8_t>(A + x * lda + y) >= p;
    if (cnt) atomicAdd(bad, cnt);
}

// entries >= p of many matrices: workgroup (x, y) scans rows x, x + gridDim.x,
// ... of matrix y and adds its count to bad[y]
struct RangeArg {
    const uint8_t* A;
    int64_t m, n, lda;
    int32_t p;
};
__global__ void __launch_bounds__(SMALL_THREADS)
k_range_many(const RangeArg* __restrict__ ds, unsigned long long* bad) {
    const RangeArg d = ds[blockIdx.y];
    unsigned long long cnt = 0;
    for (int64_t x = blockIdx.x; x < d.m; x += gridDim.x)
        for (int64_t y = threadIdx.x; y < d.n; y += SMALL_THREADS) cnt += gload<uint8_t>(d.A + x * d.lda + y) >= d.p;
    if (cnt) atomicAdd(bad + blockIdx.y, cnt);
}

// GF(2) rows packed least significant bit first in 64-bit words, unpacked to
// one byte per entry.  Thread c of a row writes the 16 entries of bits
// 16 (c mod 4) .. 16 (c mod 4) + 15 of word c / 4, as one 16-byte store when
// they lie inside the row and the destination is 16-byte aligned.
__global__ void __launch_bounds__(SMALL_THREADS)
k_unpack_gf2(const uint64_t* __restrict__ src, int64_t m, int64_t n, int64_t ldw, uint8_t* __restrict__ dst,
             int64_t ldd) {
    const int64_t chunks = (n + 15) / 16;
    for (int64_t x = blockIdx.x; x < m; x += gridDim.x) {
        uint8_t* d = dst + x * ldd;
        for (int64_t c = threadIdx.x; c < chunks; c += SMALL_THREADS) {
            const uint32_t bits = (uint32_t)(src[x * ldw + c / 4] >> (16 * (c & 3))) & 0xFFFFu;
            const int64_t y0 = c * 16;
            if (y0 + 16 <= n && (((uintptr_t)(d + y0)) & 15) == 0) {
                u32x4 v;
                for (int q = 0; q < 4; ++q) {
                    const uint32_t b = bits >> (4 * q);
                    v[q] = (b & 1u) | ((b >> 1) & 1u) << 8 | ((b >> 2) & 1u) << 16 | ((b >> 3) & 1u) << 24;
                }
                *(u32x4*)(d + y0) = v;
            } else {
                for (int q = 0; q < 16 && y0 + q < n; ++q) d[y0 + q] = (uint8_t)((bits >> q) & 1u);
            }
        }
    }
}

// ---- MAD over GF(2) on bit-packed rows, by the method of the four Russians:
// for each group of 8 rows of B (8 bits of each row of A), a table of all 256
// XOR combinations of those rows (restricted to the tile's columns) is built
// in LDS, and each row of D takes the table entry its byte of A selects.  A
// workgroup owns 256 rows (one per thread) and 1024 columns (32 dwords); the
// tables of two groups alternate, so building the next and using the current
// need one barrier per group.  Table entry e is 8 chunks of 16 bytes, chunk c
// at position (c + e) mod 8, so the lanes of a wave, which select different
// entries, spread over the banks.
constexpr int G2_THREADS = 256;
constexpr int G2_TW = 32;                      // dwords per row of the tile (1024 columns)
constexpr int G2_TABLE = 256 * G2_TW * 4;      // bytes of one table

__device__ __forceinline__ int g2_pos(int e, int c) { return e * (G2_TW * 4) + (((c + e) & 7) << 4); }

__global__ void __launch_bounds__(G2_THREADS) k_mad_gf2(Gf2MadDesc d, int tiles_n) {
    extern __shared__ __attribute__((aligned(16))) uint8_t g2s[];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * G2_THREADS;
    const int64_t w0 = (int64_t)(blockIdx.x % tiles_n) * G2_TW;   // first dword of the tile
    const int64_t nw = (d.N + 31) / 32;                            // dwords of a row of D
    const int64_t row = m0 + tid;
    const bool live = row < d.M;
    const uint32_t* A32 = (const uint32_t*)d.A;
    const uint32_t* B32 = (const uint32_t*)d.B;
    // builder role: dword w of the tile, entries 32 q .. 32 q + 31
    const int bw = tid & 31, bq = tid >> 5;
    const bool bcol = w0 + bw < nw;
    const int ngroups = (int)((d.K + 7) / 8);
    const auto build = [&](int g, uint8_t* T) {
        uint32_t br[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int64_t k = (int64_t)g * 8 + b;
            br[b] = (k < d.K && bcol) ? gload<uint32_t>(B32 + k * d.ldb * 2 + w0 + bw) : 0u;
        }
        uint32_t v = ((bq & 1) ? br[5] : 0u) ^ ((bq & 2) ? br[6] : 0u) ^ ((bq & 4) ? br[7] : 0u);
        // Gray-code order over the low five bits: one XOR per entry
#pragma unroll
        for (int l = 0; l < 32; ++l) {
            if (l) v ^= br[__builtin_ctz(l)];
            const int e = 32 * bq + (l ^ (l >> 1));
            *(uint32_t*)(T + g2_pos(e, bw >> 2) + (bw & 3) * 4) = v;
        }
    };
    uint32_t acc[G2_TW];
#pragma unroll
    for (int i = 0; i < G2_TW; ++i) acc[i] = 0;
    uint64_t aw = 0;
    if (ngroups > 0) build(0, g2s);
    __syncthreads();
    for (int g = 0; g < ngroups; ++g) {
        uint8_t* T = g2s + (g & 1) * G2_TABLE;
        if (g + 1 < ngroups) build(g + 1, g2s + ((g + 1) & 1) * G2_TABLE);
        if ((g & 7) == 0) aw = live ? gload<uint64_t>(d.A + row * d.lda + g / 8) : 0ull;
        uint32_t a = (uint32_t)(aw >> (8 * (g & 7))) & 0xffu;
        const int64_t kleft = d.K - (int64_t)g * 8;
        if (kleft < 8) a &= (1u << kleft) - 1u;            // bits of A past K - 1
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint4 t = *(const uint4*)(T + g2_pos((int)a, c));
            acc[4 * c] ^= t.x; acc[4 * c + 1] ^= t.y; acc[4 * c + 2] ^= t.z; acc[4 * c + 3] ^= t.w;
        }
        __syncthreads();
    }
    (void)A32;
    if (!live) return;
    const uint32_t* C32 = d.C ? (const uint32_t*)(d.C + row * d.ldc) : nullptr;
    uint32_t* D32 = (uint32_t*)(d.D + row * d.ldd);
#pragma unroll
    for (int i = 0; i < G2_TW; ++i) {
        const int64_t w = w0 + i;
        if (w < nw) gstore<uint32_t>(D32 + w, acc[i] ^ (C32 ? gload<uint32_t>(C32 + w) : 0u));
    }
}

// rows whose last word has a bit set past column n - 1 (n not a multiple of 64)
__global__ void __launch_bounds__(SMALL_THREADS)
k_gf2_pad(const uint64_t* __restrict__ src, int64_t m, int64_t n, int64_t ldw, unsigned long long* bad) {
    const uint64_t mask = ~((1ull << (n & 63)) - 1);
    unsigned long long cnt = 0;
    for (int64_t x = blockIdx.x * SMALL_THREADS + threadIdx.x; x < m; x += (int64_t)gridDim.x * SMALL_THREADS)
        cnt += (src[x * ldw + n / 64] & mask) != 0;
    if (cnt) atomicAdd(bad, cnt);
}

// The fixed workspace of the allocation-free ECH entry point, a plain device
// array: host code must not pass this name to a kernel (on the host it names a
// stand-in, not the device address); it uses the address hipGetSymbolAddress
// returns at initialisation.
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

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
        // lanes 1, 2 and 3 are created when first used (lane_stream): a
        // process's streams share its few hardware queues, and an instance
        // whose problems never use them (single-block problems, input copies)
        // should not take a share
        if (hipFuncSetAttribute((const void*)k_ech_panel<DescArg<EchDesc, ECH_ARG_CAP>>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)echp_lds_bytes(ECHP_MAX_ROWS)) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_ech_panel<DescPtr<EchDesc>>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)echp_lds_bytes(ECHP_MAX_ROWS)) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_gemm_modp<2, GemmArgSrc>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)GemmCfg<2>::lds_bytes()) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_gemm_modp<2, GemmPtrSrc>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)GemmCfg<2>::lds_bytes()) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_gemm_modp<4, GemmArgSrc>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)GemmCfg<4>::lds_bytes()) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_gemm_modp<4, GemmPtrSrc>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)GemmCfg<4>::lds_bytes()) != hipSuccess) {
            if (err) *err = "cannot reserve LDS for the kernels";
            return false;
        }
        if (hipFuncSetAttribute((const void*)k_mad_gf2, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * G2_TABLE) !=
            hipSuccess) {
            if (err) *err = "cannot reserve LDS for the GF(2) kernel";
            return false;
        }
        // the LDS-resident ECH takes up to 160 KB per workgroup where the device allows it
        echs_lds_max_ = 160 * 1024;
        if (hipFuncSetAttribute((const void*)k_ech_lds<DescArg<EchDesc, ECH_ARG_CAP>>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)echs_lds_max_) != hipSuccess ||
            hipFuncSetAttribute((const void*)k_ech_lds<DescPtr<EchDesc>>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)echs_lds_max_) != hipSuccess) {
            (void)hipGetLastError();
            echs_lds_max_ = 64 * 1024;
        }
        no_lds_ech_ = getenv("GFECH_ECH_NO_LDS") != nullptr;
        const char* gg = getenv("GFECH_GEMM_GROUP");
        gemm_group_ = gg ? std::max(1, std::min(64, atoi(gg))) : 4;
        const char* gw = getenv("GFECH_GEMM_WIDE");
        gemm_wide_ = !(gw && gw[0] == '0');
        // the device address of the fixed workspace on this device (the one
        // current now, which every later call of this backend uses)
        if (hipGetSymbolAddress((void**)&fixed_scratch_, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            fixed_scratch_ = nullptr;
        }
        return true;
    }
    uint8_t* fixed_scratch() override { return fixed_scratch_; }

    const char* name() const override { return "hip-gfx950"; }

    // alloc and release may run outside the instance's lock (a result freed by
    // another thread); the memory cache has a lock of its own
    void* alloc(size_t bytes) override {
        std::lock_guard<std::mutex> lk(cache_mu_);
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
        std::lock_guard<std::mutex> lk(cache_mu_);
        auto it = sizes_.find(p);
        if (it == sizes_.end()) return;
        free_.insert({it->second, p});
        sizes_.erase(it);
    }
    void trim() {
        sync_all();
        for (auto& kv : free_) hipFree(kv.second);
        free_.clear();
    }
    void zero(void* p, size_t bytes) override {
        if (bytes) HIP_OK(hipMemsetAsync(p, 0, bytes, stream_));
    }
    // memory transfers run on lane 0 (stream_); kernels on the current lane (cur_)
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
    void sync() override { sync_all(); }
    void sync_lane0() override { HIP_OK(hipStreamSynchronize(stream_)); }
    // pinned host memory the device writes directly: no copy, only a wait for lane 0
    int32_t* counts_buffer(size_t n) override {
        if (n > counts_cap_) {
            sync_all();
            pending_.clear();
            if (counts_host_) (void)hipHostFree(counts_host_);
            counts_host_ = nullptr;
            counts_dev_ = nullptr;
            counts_cap_ = 0;
            void* h = nullptr;
            if (hipHostMalloc(&h, sizeof(int32_t) * n, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            void* d = nullptr;
            if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipHostFree(h);
                return nullptr;
            }
            counts_host_ = (int32_t*)h;
            counts_dev_ = (int32_t*)d;
            counts_cap_ = n;
        }
        return counts_dev_;
    }
    // The ECH kernels write each pivot count straight into the pinned counts
    // buffer, once, with its final value.  ech() sets the slots it launches for
    // to -1 first; read_counts then polls those slots instead of sleeping in a
    // stream synchronisation (whose wake-up came tens of microseconds after
    // the kernel on this chain), asking the stream every 64 polls, so that a
    // failed launch or a finished stream ends the wait.  The work queued after
    // the ECH stays ordered behind it on its stream.
    void read_counts(int32_t* host, const int32_t* counts, size_t n) override {
        if (counts == counts_dev_ && n <= counts_cap_) {
            if (pending_.empty()) HIP_OK(hipStreamSynchronize(stream_));
            else wait_pending();
            for (size_t k = 0; k < n; ++k) host[k] = __atomic_load_n(counts_host_ + k, __ATOMIC_ACQUIRE);
            return;
        }
        HIP_OK(hipStreamSynchronize(stream_));
        download(host, counts, sizeof(int32_t) * n);
    }
    void wait_pending() {
        for (uint64_t spin = 1;; ++spin) {
            bool ready = true;
            for (size_t k : pending_)
                if (__atomic_load_n(counts_host_ + k, __ATOMIC_ACQUIRE) < 0) {
                    ready = false;
                    break;
                }
            if (ready) break;
            if ((spin & 63) == 0) {
                const hipError_t q = hipStreamQuery(stream_);
                if (q == hipErrorNotReady) continue;
                HIP_OK(q);
                // the stream is idle: every count it was going to write is there
                for (size_t k : pending_)
                    if (__atomic_load_n(counts_host_ + k, __ATOMIC_ACQUIRE) < 0)
                        note_error(hipErrorUnknown, "pivot count missing");
                break;
            }
            __builtin_ia32_pause();
        }
        pending_.clear();
    }
    void release_counts(int32_t*) override {}
    void set_stream(void* s) override {
        stream_ = (hipStream_t)s;
        cur_ = stream_;
    }
    void set_lane(int lane) override { cur_ = lane_stream(lane); }
    // lanes 1, 2 and 3: streams of their own at the default priority,
    // non-blocking (they never synchronise implicitly with the legacy default
    // stream), created on first use
    hipStream_t lane_stream(int lane) {
        if (lane < 1 || lane > 3) return stream_;
        hipStream_t& s = lanes_[lane - 1];
        if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            note_error(hipErrorOutOfMemory, "stream creation");
            s = nullptr;
            return stream_;
        }
        return s;
    }
    void* create_stream() override {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return st;
    }
    void destroy_stream(void* st) override {
        if (!st) return;
        sync_all();
        HIP_OK(hipStreamSynchronize((hipStream_t)st));
        HIP_OK(hipStreamDestroy((hipStream_t)st));
    }
    int mark(int lane) override {
        hipEvent_t e = nullptr;
        if (!mark_pool_.empty()) {
            e = mark_pool_.back();
            mark_pool_.pop_back();
        } else {
            HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        hipStream_t s = lane_stream(lane);
        HIP_OK(hipEventRecord(e, s));
        marks_.push_back(e);
        mark_streams_.push_back(s);
        return mark_base_ + (int)marks_.size() - 1;
    }
    // A stream-wait costs the host about ten microseconds, so the waits that
    // order nothing are left out: on a mark of the waiting stream itself, on a
    // mark at or before one of the same stream this stream already waited for
    // (marks of one stream complete in order), and on a mark already reached.
    void wait_mark(int lane, int m) override {
        // marks below mark_base_ were passed by a full synchronisation already
        if (m < mark_base_ || m - mark_base_ >= (int)marks_.size()) return;
        const hipStream_t w = lane_stream(lane), src = mark_streams_[m - mark_base_];
        if (w == src) return;
        Waited* slot = nullptr;
        for (Waited& x : waited_)
            if (x.waiter == w && x.source == src) slot = &x;
        if (slot && slot->mark >= m) return;
        if (!slot) {
            waited_.push_back({w, src, -1});
            slot = &waited_.back();
        }
        slot->mark = m;
        const hipError_t q = hipEventQuery(marks_[m - mark_base_]);
        if (q == hipSuccess) return;
        if (q != hipErrorNotReady) note_error(q, "hipEventQuery");
        HIP_OK(hipStreamWaitEvent(w, marks_[m - mark_base_], 0));
    }
    int error() const override { return err_; }

    // The 256 x 256 tile (eight waves) for every product; GFECH_GEMM_WIDE=0
    // takes the 256 x 128 tile (four waves, two workgroups per compute unit)
    // instead.  Measured on the 40000 x 40000 GF(7) solve: 103.9 ms against
    // 105.9 ms; the isolated layer launch 0.556 ms against 0.635 ms; the
    // batch of 4096 small matrices 53.9K solves/s against 47.5K; the wide
    // tile for products of at least 1024 columns and the narrow one for the
    // rest (two launches): 110.7 ms.
    void gemm(const std::vector<GemmDesc>& ds) override {
        std::vector<GemmDesc> d;
        for (const GemmDesc& g : ds)
            if (g.M > 0 && g.N > 0) d.push_back(g);
        if (d.empty()) return;
        if (gemm_wide_) gemm_launch<4>(d);
        else gemm_launch<2>(d);
    }
    template <int WN>
    void gemm_launch(const std::vector<GemmDesc>& ds) {
        using GC = GemmCfg<WN>;
        std::vector<GemmDesc> d;
        std::vector<GemmTileMap> maps;
        int64_t tiles = 0;
        for (const GemmDesc& g : ds) {
            if (g.K > 65536) { note_error(hipErrorInvalidValue, "gemm K > 65536"); return; }
            GemmTileMap t;
            t.tiles_n = (g.N + GC::TN - 1) / GC::TN;
            t.first_tile = (int32_t)tiles;
            tiles += (int64_t)((g.M + TM - 1) / TM) * t.tiles_n;
            d.push_back(g);
            maps.push_back(t);
        }
        if (d.empty()) return;
        if (tiles > INT32_MAX) { note_error(hipErrorInvalidValue, "too many gemm tiles"); return; }
        launch_mac_ = 0;
        for (const GemmDesc& g : d) launch_mac_ += (double)g.M * g.N * g.K;
        const unsigned grid = (unsigned)tiles;
        if (d.size() <= (size_t)GEMM_ARG_CAP) {
            GemmArgSrc a;
            a.n = (int)d.size();
            a.group = gemm_group_;
            for (size_t i = 0; i < d.size(); ++i) { a.m[i] = maps[i]; a.d[i] = d[i]; }
            go(0, k_gemm_modp<WN, GemmArgSrc>, dim3(grid), dim3(GC::THREADS), GC::lds_bytes(), a);
        } else {
            // one upload: the tile maps, then the descriptors (256-byte aligned)
            const size_t mb = (maps.size() * sizeof(GemmTileMap) + 255) & ~(size_t)255;
            std::vector<uint8_t> blob(mb + d.size() * sizeof(GemmDesc));
            memcpy(blob.data(), maps.data(), maps.size() * sizeof(GemmTileMap));
            memcpy(blob.data() + mb, d.data(), d.size() * sizeof(GemmDesc));
            const uint8_t* dev = (const uint8_t*)put(blob.data(), blob.size());
            GemmPtrSrc a;
            a.n = (int)d.size();
            a.group = gemm_group_;
            a.m = (const GemmTileMap*)dev;
            a.d = (const GemmDesc*)(dev + mb);
            go(0, k_gemm_modp<WN, GemmPtrSrc>, dim3(grid), dim3(GC::THREADS), GC::lds_bytes(), a);
        }
        HIP_OK(hipGetLastError());
    }

    // launch `kernel` over descriptors: up to CAP by value, otherwise uploaded
    template <int CAP, typename D, typename KArg, typename KPtr>
    void launch_descs(const D* ds, size_t cnt, KArg karg, KPtr kptr, dim3 grid, dim3 block, size_t shm, int kind) {
        if (cnt <= (size_t)CAP) {
            DescArg<D, CAP> a;
            for (size_t i = 0; i < cnt; ++i) a.d[i] = ds[i];
            go(kind, karg, grid, block, shm, a);
        } else {
            DescPtr<D> a;
            a.p = (const D*)put(ds, cnt * sizeof(D));
            go(kind, kptr, grid, block, shm, a);
        }
        HIP_OK(hipGetLastError());
    }

    void ech(const std::vector<EchDesc>& ds) override {
        if (ds.empty()) return;
        // the slots these ECHs write in the pinned counts buffer: -1 until written
        for (const EchDesc& e : ds) {
            if (e.rcount >= counts_dev_ && e.rcount < counts_dev_ + counts_cap_) {
                const size_t k = (size_t)(e.rcount - counts_dev_);
                __atomic_store_n(counts_host_ + k, -1, __ATOMIC_RELEASE);
                pending_.push_back(k);
            }
        }
        // blocks of at most 256 rows over p <= 46 whose working matrix fits in
        // LDS: k_ech_lds; the others below
        std::vector<EchDesc> lds, rest;
        size_t shm_lds = 0;
        for (const EchDesc& e : ds) {
            const size_t need = echs_lds_bytes(e.rows, e.cols);
            if (e.rows <= ECHS_MAX_ROWS && e.p <= ECHS_MAX_P && need <= echs_lds_max_ && !no_lds_ech_) {
                lds.push_back(e);
                shm_lds = std::max(shm_lds, need);
            } else {
                rest.push_back(e);
            }
        }
        // largest blocks first: the hardware hands out workgroups in order, so
        // the longest ones start first and the launch ends with short ones
        const auto larger = [](const EchDesc& a, const EchDesc& b) {
            return (int64_t)a.rows * a.cols > (int64_t)b.rows * b.cols;
        };
        std::stable_sort(lds.begin(), lds.end(), larger);
        std::stable_sort(rest.begin(), rest.end(), larger);
        for (size_t off = 0; off < lds.size(); off += 65535) {
            const size_t cnt = std::min<size_t>(65535, lds.size() - off);
            launch_descs<ECH_ARG_CAP>(lds.data() + off, cnt, k_ech_lds<DescArg<EchDesc, ECH_ARG_CAP>>,
                                      k_ech_lds<DescPtr<EchDesc>>, dim3((unsigned)cnt), dim3(ECHS_THREADS), shm_lds, 1);
        }
        if (!rest.empty()) ech_global(rest);
    }
    void ech_global(const std::vector<EchDesc>& ds) {
        int maxrows_all = 0;
        for (const EchDesc& e : ds) maxrows_all = std::max(maxrows_all, e.rows);
        if (maxrows_all <= ECHP_MAX_ROWS && !getenv("GFECH_ECH_SIMPLE")) {
            int threads = std::max(64, (maxrows_all + 63) / 64 * 64);
            size_t shm = echp_lds_bytes(maxrows_all);
            for (size_t off = 0; off < ds.size(); off += 65535) {
                const size_t cnt = std::min<size_t>(65535, ds.size() - off);
                launch_descs<ECH_ARG_CAP>(ds.data() + off, cnt, k_ech_panel<DescArg<EchDesc, ECH_ARG_CAP>>,
                                          k_ech_panel<DescPtr<EchDesc>>, dim3((unsigned)cnt), dim3(threads), shm, 1);
            }
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
        for (size_t off = 0; off < ds.size(); off += 65535) {
            const size_t cnt = std::min<size_t>(65535, ds.size() - off);
            launch_descs<ECH_ARG_CAP>(ds.data() + off, cnt, k_ech<DescArg<EchDesc, ECH_ARG_CAP>>,
                                      k_ech<DescPtr<EchDesc>>, dim3((unsigned)cnt), dim3(ECH_THREADS), shm, 1);
        }
    }

    template <typename D, typename KArg, typename KPtr>
    void small(const std::vector<D>& ds, KArg karg, KPtr kptr, int64_t (*work)(const D&)) {
        if (ds.empty()) return;
        int64_t mx = 1;
        for (const D& x : ds) mx = std::max(mx, work(x));
        int64_t bx = std::min<int64_t>((mx + SMALL_THREADS - 1) / SMALL_THREADS, 4096);
        for (size_t off = 0; off < ds.size(); off += 65535) {
            size_t cnt = std::min<size_t>(65535, ds.size() - off);
            launch_descs<SMALL_ARG_CAP>(ds.data() + off, cnt, karg, kptr, dim3((unsigned)bx, (unsigned)cnt),
                                        dim3(SMALL_THREADS), 0, 2);
        }
    }

    void gather(const std::vector<GatherDesc>& ds) override {
        // one block per row (up to the cap); the work function counts rows x threads
        small<GatherDesc>(ds, k_gather<DescArg<GatherDesc, SMALL_ARG_CAP>>, k_gather<DescPtr<GatherDesc>>,
                          [](const GatherDesc& g) -> int64_t { return (int64_t)g.rows * SMALL_THREADS; });
    }
    void fill(const std::vector<FillDesc>& ds) override {
        small<FillDesc>(ds, k_fill<DescArg<FillDesc, SMALL_ARG_CAP>>, k_fill<DescPtr<FillDesc>>,
                        [](const FillDesc& f) -> int64_t {
                            return f.dcol ? (int64_t)f.rows : (int64_t)f.rows * SMALL_THREADS;
                        });
    }
    void lists(const std::vector<ListDesc>& ds) override {
        small<ListDesc>(ds, k_lists<DescArg<ListDesc, SMALL_ARG_CAP>>, k_lists<DescPtr<ListDesc>>,
                        [](const ListDesc& l) -> int64_t { return std::max(l.npick, l.nkeep); });
    }
    void sort(const std::vector<SortDesc>& ds) override {
        small<SortDesc>(ds, k_sort<DescArg<SortDesc, SMALL_ARG_CAP>>, k_sort<DescPtr<SortDesc>>,
                        [](const SortDesc& s) -> int64_t { return (int64_t)s.n; });
    }

    int64_t count_out_of_range(const uint8_t* A, int64_t m, int64_t n, int64_t lda, int32_t p) override {
        HIP_OK(hipMemsetAsync(counter_, 0, 8, stream_));
        int64_t bx = std::min<int64_t>(m, 8192);
        hipLaunchKernelGGL(k_range, dim3((unsigned)std::max<int64_t>(bx, 1)), dim3(SMALL_THREADS), 0, stream_, A, m,
                           n, lda, p, (unsigned long long*)counter_);
        HIP_OK(hipGetLastError());
        unsigned long long bad = 0;
        download(&bad, counter_, 8);
        return err_ ? -1 : (int64_t)bad;
    }

    void count_out_of_range_many(const std::vector<RangeDesc>& ds, std::vector<int64_t>& bad) override {
        bad.assign(ds.size(), 0);
        if (ds.empty()) return;
        // descriptors and counters in one device buffer: the descriptors are
        // uploaded, the counters zeroed by the same copy
        const size_t nd = ds.size();
        std::vector<uint8_t> blob(nd * sizeof(RangeArg) + nd * 8, 0);
        int64_t mmax = 1;
        for (size_t t = 0; t < nd; ++t) {
            RangeArg a{ds[t].A, ds[t].m, ds[t].n, ds[t].lda, ds[t].p};
            memcpy(blob.data() + t * sizeof(RangeArg), &a, sizeof(a));
            mmax = std::max(mmax, ds[t].m);
        }
        uint8_t* dev = (uint8_t*)alloc(blob.size());
        if (!dev) {
            Backend::count_out_of_range_many(ds, bad);
            return;
        }
        upload(dev, blob.data(), blob.size());
        unsigned long long* cnt = (unsigned long long*)(dev + nd * sizeof(RangeArg));
        for (size_t off = 0; off < nd; off += 65535) {
            const size_t c = std::min<size_t>(65535, nd - off);
            hipLaunchKernelGGL(k_range_many, dim3((unsigned)std::min<int64_t>(mmax, 64), (unsigned)c),
                               dim3(SMALL_THREADS), 0, stream_, (const RangeArg*)dev + off, cnt + off);
        }
        HIP_OK(hipGetLastError());
        std::vector<unsigned long long> h(nd);
        download(h.data(), cnt, nd * 8);
        release(dev);
        for (size_t t = 0; t < nd; ++t) bad[t] = err_ ? -1 : (int64_t)h[t];
    }
    void unpack_gf2(const uint64_t* src, int64_t m, int64_t n, int64_t ldw, uint8_t* dst, int64_t ldd) override {
        if (m <= 0 || n <= 0) return;
        hipLaunchKernelGGL(k_unpack_gf2, dim3((unsigned)std::min<int64_t>(m, 65535)), dim3(SMALL_THREADS), 0, stream_,
                           src, m, n, ldw, dst, ldd);
        HIP_OK(hipGetLastError());
    }
    void mad_gf2(const Gf2MadDesc& d) override {
        if (d.M <= 0 || d.N <= 0) return;
        const int64_t nw = (d.N + 31) / 32;
        const int64_t tn = (nw + G2_TW - 1) / G2_TW, tm = (d.M + G2_THREADS - 1) / G2_THREADS;
        if (tn * tm > INT32_MAX) { note_error(hipErrorInvalidValue, "gf2 mad too large"); return; }
        launch_mac_ = (double)d.M * d.N * d.K;
        go(0, k_mad_gf2, dim3((unsigned)(tn * tm)), dim3(G2_THREADS), (size_t)(2 * G2_TABLE), d, (int)tn);
        HIP_OK(hipGetLastError());
    }
    int64_t count_gf2_pad(const uint64_t* src, int64_t m, int64_t n, int64_t ldw) override {
        if (m <= 0 || n <= 0 || n % 64 == 0) return 0;
        HIP_OK(hipMemsetAsync(counter_, 0, 8, stream_));
        const int64_t bx = std::min<int64_t>((m + SMALL_THREADS - 1) / SMALL_THREADS, 4096);
        hipLaunchKernelGGL(k_gf2_pad, dim3((unsigned)bx), dim3(SMALL_THREADS), 0, stream_, src, m, n, ldw,
                           (unsigned long long*)counter_);
        HIP_OK(hipGetLastError());
        unsigned long long bad = 0;
        download(&bad, counter_, 8);
        return err_ ? -1 : (int64_t)bad;
    }

    void set_profile(int level) override { prof_ = level; }
    Profile take_profile() override {
        Profile pr;
        sync_all();
        for (auto& ev : evs_) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
                pr.ms[ev.kind] += ms;
                pr.launches[ev.kind] += 1;
                pr.mac[ev.kind] += ev.mac;
            }
            pool_.push_back(ev.a);
            pool_.push_back(ev.b);
        }
        evs_.clear();
        return pr;
    }

private:
    struct Ev { hipEvent_t a, b; int kind; double mac; };
    // profile level 3 times a pseudo-random quarter of the MAD launches (a
    // fixed stride would beat against the period of a layer's launches):
    // the finalizer of MurmurHash3 on the launch number
    static bool sample_quarter(uint64_t x) {
        x ^= x >> 33;
        x *= 0xff51afd7ed558ccdull;
        x ^= x >> 33;
        x *= 0xc4ceb9fe1a85ec53ull;
        x ^= x >> 33;
        return (x & 3) == 0;
    }
    double launch_mac_ = 0;     // multiply-adds of the MAD launch being issued
    int64_t mad_seq_ = 0;       // MAD launches issued at profile level 3
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
    // Launch on the current lane.  When launches of this kind are profiled
    // (level 1: every launch; level 2: MAD launches only, kind 0) the launch
    // carries a start and a stop event that take the dispatch's own begin and
    // end timestamps, so the recorded time is the kernel's execution alone.
    template <typename F, typename... Args>
    void go(int kind, F kernel, dim3 grid, dim3 block, size_t shm, Args... args) {
        const bool timed = prof_ == 1 || (prof_ >= 2 && kind == 0 && (prof_ == 2 || sample_quarter(mad_seq_++)));
        if (!timed) {
            hipLaunchKernelGGL(kernel, grid, block, shm, cur_, args...);
            return;
        }
        hipEvent_t a = new_event(), b = new_event();
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, cur_, a, b, 0, args...);
        evs_.push_back({a, b, kind, kind == 0 ? launch_mac_ : 0.0});
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
            sync_all();   // earlier copies out of the ring, and the kernels reading them, are done
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
        HIP_OK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, cur_));   // ordered before the launch reading it
        return d;
    }
    // every lane drained; the marks can be reused
    void sync_all() {
        for (hipStream_t s : lanes_)
            if (s) HIP_OK(hipStreamSynchronize(s));
        HIP_OK(hipStreamSynchronize(stream_));
        for (hipEvent_t e : marks_) mark_pool_.push_back(e);
        mark_base_ += (int)marks_.size();
        if (mark_base_ > (1 << 30)) mark_base_ = 0;
        marks_.clear();
        mark_streams_.clear();
        waited_.clear();
    }

    hipStream_t stream_ = nullptr;   // lane 0: the caller's stream
    hipStream_t lanes_[3] = {nullptr, nullptr, nullptr};   // lanes 1, 2 and 3 (created on first use)
    hipStream_t cur_ = nullptr;      // the lane kernels go to
    std::vector<hipEvent_t> marks_, mark_pool_;
    std::vector<hipStream_t> mark_streams_;   // the stream each of marks_ was recorded on
    struct Waited { hipStream_t waiter, source; int mark; };
    std::vector<Waited> waited_;     // since the last full synchronisation: the latest mark of
                                     // `source` that `waiter` waits for
    int32_t* counts_host_ = nullptr;   // counts_buffer(): host view
    int32_t* counts_dev_ = nullptr;    // and device view
    std::vector<size_t> pending_;      // slots of counts_host_ an ECH queued since the last read will write
    size_t counts_cap_ = 0;
    int mark_base_ = 0;              // id of marks_[0]
    size_t echs_lds_max_ = 0;        // LDS the LDS-resident ECH may use
    bool no_lds_ech_ = false;
    int gemm_group_ = 4;             // tile rows per group of the MAD tile order (measured: 4)
    bool gemm_wide_ = true;          // 256 x 256 MAD tiles (GFECH_GEMM_WIDE=0: 256 x 128)
    void* ring_host_ = nullptr;
    void* ring_dev_ = nullptr;
    size_t ring_off_ = 0;
    void* counter_ = nullptr;
    uint8_t* fixed_scratch_ = nullptr;   // device address of `scratch`
    int err_ = 0;
    int num_cu_ = 0;
    int prof_ = 0;
    std::vector<Ev> evs_;
    std::vector<hipEvent_t> pool_;
    std::mutex cache_mu_;               // sizes_ and free_
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

// Further instances for the server's size classes, kept in a pool: an
// instance is never destroyed (results refer to the instance that made them),
// a released one is handed out again.
namespace {
std::mutex g_pool_mu;
std::vector<HipBackend*> g_pool;
}  // namespace

Backend* backend_acquire(std::string* err) {
    if (!backend_instance(err)) return nullptr;          // the device checks, once
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (!g_pool.empty()) {
            HipBackend* b = g_pool.back();
            g_pool.pop_back();
            return b;
        }
    }
    HipBackend* b = new HipBackend();
    std::string e;
    if (!b->init(&e)) {
        delete b;
        if (err) *err = e;
        return nullptr;
    }
    return b;
}

void backend_release(Backend* be) {
    if (!be) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(static_cast<HipBackend*>(be));
}

}  // namespace gfech
