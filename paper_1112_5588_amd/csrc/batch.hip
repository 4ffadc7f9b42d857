// Many pJDS products at once: y_m = A_m x_m for a batch of matrices of very different sizes.
//
// Three execution modes share one handle:
//  * PJDS_BATCH_PERSISTENT: a single launch of a persistent kernel.  The rows of all members
//    are cut into tiles of up to `groups_per_tile` wave groups (64 sorted rows each); the
//    tiles are ordered member by member, largest member first, and every wave pulls the
//    next tile from one device counter until the table is exhausted (every wave then exits).  A small
//    fill kernel resets the counter in front of it.  Both kernels are captured once in a
//    HIP graph; a launch replays it.
//  * pjds_batch_create_xlds: the persistent kernel with x staged in LDS.  Workgroups (not
//    waves) pull the tiles; a workgroup copies the x range its tile's sort windows cover, plus
//    a halo on each side, into LDS, then its waves pull the tile's wave groups from an LDS
//    counter and read x from LDS wherever the column falls in the staged range.
//  * PJDS_BATCH_GRAPH: one pjds_spmv launch per member, captured in a HIP graph.
//  * PJDS_BATCH_DIRECT: one pjds_spmv launch per member, issued on the stream each time.
// Rows are never split here (no long-row workspace); results equal pjds_spmv's bit for bit
// when the member was planned without long-row splitting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"
#include "device.h"

namespace pjds {
namespace {

constexpr int kBlock = 256;
#ifndef PJDS_UNROLL
#define PJDS_UNROLL 8
#endif
constexpr int kUnroll = PJDS_UNROLL;
static_assert(kUnroll == 4 || kUnroll == 8, "the clamped tail covers remainders below 8");

struct Member {                    // device-side descriptor of one batch member
    const int32_t *row_len;
    const int64_t *offsets;
    const int32_t *col_p;
    const void *val_p;
    const int32_t *perm;
    const void *x;
    void *y;
    int64_t n_rows, n_pad;
    int64_t n_cols;
    int64_t window;                // sort window in rows (n_pad for a global sort)
};

struct Tile {                      // wave groups [g0, g1) of member m
    int32_t m, g0, g1, pad;
};

// Accesses through the member pointers.  Those pointers are read from device memory, so the
// compiler takes them as generic and issues flat loads, which count on the LDS counter as well.
// With G they load and store through address-space-1 pointers instead (global loads).  The
// kernel that reads x through the caches takes that form (0.7-1.4% faster); the one that reads
// x from LDS keeps the generic form, which measured faster there.
template <bool G, class T>
__device__ __forceinline__ T m_ld(const T *p) {
    typedef __attribute__((address_space(1))) const T GT;
    if constexpr (G) return *(const GT *)p;
    else return *p;
}
template <bool G, class T>
__device__ __forceinline__ T m_ld_nt(const T *p) {               // streamed once
    typedef __attribute__((address_space(1))) const T GT;
    if constexpr (G) return __builtin_nontemporal_load((const GT *)p);
    else return __builtin_nontemporal_load(p);
}
template <bool G, class T>
__device__ __forceinline__ void m_st(T *p, T v) {
    typedef __attribute__((address_space(1))) T GT;
    if constexpr (G) *(GT *)p = v;
    else *p = v;
}

// x gathered from global memory
template <class T>
struct XGlobal {
    static constexpr bool kTyped = true;
    const T *x;
    __device__ __forceinline__ T operator()(int32_t c) const { return m_ld<true>(x + c); }
};

// x[lo, lo + n) staged in LDS; columns outside that range read global memory
template <class T>
struct XStaged {
    static constexpr bool kTyped = false;
    const T *lds;
    const T *x;
    uint32_t lo, n;
    __device__ __forceinline__ T operator()(int32_t c) const {
        return staged_or_global<T>(lds, uint32_t(c) - lo, n, 1, x, c);
    }
};

// U entries from jb; with CLAMP, steps at or past m re-read step m - 1 and are masked (one
// round trip for a ragged tail, no load past the longest row).
template <int U, bool CLAMP, class T, bool JD, int BR, class XA>
__device__ __forceinline__ void steps(T &acc, int jb, int m, int len, int64_t base, int64_t base_lead,
                                      const int64_t *__restrict__ off, const int32_t *__restrict__ col_p,
                                      const T *__restrict__ val_p, const XA &x) {
    constexpr bool G = XA::kTyped;
    T v[U];
    int32_t c[U];
    int64_t a[U];                                      // indices first, then values
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = CLAMP ? min(jb + u, m - 1) : jb + u;
        const int64_t b = j < len ? base : base_lead;   // lead row: an entry at every such j
        a[u] = JD ? m_ld<G>(off + j) + b : b + int64_t(j) * BR;
        c[u] = m_ld_nt<G>(col_p + a[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = m_ld_nt<G>(val_p + a[u]);
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x(c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const T s = __builtin_fma(v[u], xv[u], acc);
        acc = (jb + u < len && (!CLAMP || jb + u < m)) ? s : acc;
    }
}

// One wave group of one member: Listing 2 over 64 sorted rows, same arithmetic order as
// pjds_spmv (entries in stored order, one FMA each).
template <class T, bool JD, int BR, class XA>
__device__ __forceinline__ void wave_group(const Member &M, int64_t g, bool y_perm, const XA &x) {
    constexpr bool G = XA::kTyped;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = g * kWave + lane;
    int len = m_ld<G>(M.row_len + (i < M.n_pad ? i : M.n_pad - 1));   // clamped, then masked
    const int64_t base = JD ? i : m_ld<G>(M.offsets + (i < M.n_pad ? i : M.n_pad - 1) / BR) + (i % BR);
    if (i >= M.n_pad) len = 0;
    const int m = __builtin_amdgcn_readfirstlane(len);
    T acc = T(0);
    if (m > 0) {
        const int64_t base_lead = wave_first(base);
        const T *val_p = static_cast<const T *>(M.val_p);
        int jb = 0;
        for (; jb + kUnroll <= m; jb += kUnroll)
            steps<kUnroll, false, T, JD, BR>(acc, jb, m, len, base, base_lead, M.offsets, M.col_p, val_p, x);
        const int r = m - jb;
        if (r > 4) steps<8, true, T, JD, BR>(acc, jb, m, len, base, base_lead, M.offsets, M.col_p, val_p, x);
        else if (r > 2) steps<4, true, T, JD, BR>(acc, jb, m, len, base, base_lead, M.offsets, M.col_p, val_p, x);
        else if (r == 2) steps<2, false, T, JD, BR>(acc, jb, m, len, base, base_lead, M.offsets, M.col_p, val_p, x);
        else if (r == 1) steps<1, false, T, JD, BR>(acc, jb, m, len, base, base_lead, M.offsets, M.col_p, val_p, x);
    }
    if (i < M.n_rows) m_st<G>(static_cast<T *>(M.y) + (y_perm ? i : m_ld<G>(M.perm + i)), acc);
}

// The same wave group with two register sets of U steps in turn: the next group's loads go
// out before this group's FMAs, steps at or past m re-read step m - 1 and are masked (no load
// past the longest row).  Same FMAs in the same order per row as wave_group.  It holds about
// twice the registers, which pays where x comes through the caches (more gathers in flight per
// wave) and not in the staged kernel, where it costs resident waves.
template <class T, bool JD, int BR, class XA>
__device__ __forceinline__ void wave_group_pipe(const Member &M, int64_t g, bool y_perm, const XA &x) {
    constexpr int U = kUnroll;
    constexpr bool G = XA::kTyped;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = g * kWave + lane;
    int len = m_ld<G>(M.row_len + (i < M.n_pad ? i : M.n_pad - 1));   // clamped, then masked
    const int64_t base = JD ? i : m_ld<G>(M.offsets + (i < M.n_pad ? i : M.n_pad - 1) / BR) + (i % BR);
    if (i >= M.n_pad) len = 0;
    const int m = __builtin_amdgcn_readfirstlane(len);
    T acc = T(0);
    if (m > 0) {
        const int64_t base_lead = wave_first(base);
        const T *val_p = static_cast<const T *>(M.val_p);
        const int64_t *__restrict__ off = M.offsets;
        const int32_t *__restrict__ col_p = M.col_p;
        T v[2][U];
        int32_t c[2][U];
        auto load = [&](int jb, int set) {
            int64_t a[U];                              // indices first, then values
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(jb + u, m - 1);
                const int64_t b = j < len ? base : base_lead;   // lead row: an entry at every such j
                a[u] = JD ? m_ld<G>(off + j) + b : b + int64_t(j) * BR;
                c[set][u] = m_ld_nt<G>(col_p + a[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) v[set][u] = m_ld_nt<G>(val_p + a[u]);
        };
        auto group = [&](int jb, int set) {
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x(c[set][u]);
            if (jb + U < m) load(jb + U, set ^ 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const T s = __builtin_fma(v[set][u], xv[u], acc);
                acc = (jb + u < len && jb + u < m) ? s : acc;
            }
        };
        load(0, 0);
        for (int jb = 0; jb < m; jb += 2 * U) {
            group(jb, 0);
            if (jb + U < m) group(jb + U, 1);
        }
    }
    if (i < M.n_rows) m_st<G>(static_cast<T *>(M.y) + (y_perm ? i : m_ld<G>(M.perm + i)), acc);
}

// Two adjacent rows per lane (rows i, i + 1 of wave groups g and g + 1, i even): their slots
// are neighbours at every step, so one 2-wide load brings both values and one both indices.
// Row i is the longer, so lane 0's pair serves lanes that are done.  Same FMAs in the same
// order per row as wave_group.
typedef int32_t Int2 __attribute__((ext_vector_type(2)));

template <class T, bool JD, int BR, class XA>
__device__ __forceinline__ void wave_group_pair(const Member &M, int64_t g, bool y_perm, const XA &x) {
    typedef typename VecOf<T, 2>::type V2;
    constexpr bool G = XA::kTyped;
    constexpr int U = 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = g * kWave + 2 * lane;
    const int64_t ia = i < M.n_pad ? i : M.n_pad - 2;
    Int2 len = m_ld<G>(reinterpret_cast<const Int2 *>(M.row_len + ia));   // clamped, then masked
    if (i >= M.n_pad) len = Int2{0, 0};
    const int64_t base = JD ? ia : m_ld<G>(M.offsets + ia / BR) + (ia % BR);
    const int m = __builtin_amdgcn_readfirstlane(int(len.x));
    T a0 = T(0), a1 = T(0);
    if (m > 0) {
        const int64_t base_lead = wave_first(base);
        const T *val_p = static_cast<const T *>(M.val_p);
        const int64_t *__restrict__ off = M.offsets;
        const int32_t *__restrict__ col_p = M.col_p;
        // two register sets of U steps in turn: the next group's loads go out before this
        // group's FMAs; steps at or past m re-read step m - 1 and are masked
        V2 v[2][U];
        Int2 c[2][U];
        auto load = [&](int jb, int set) {
            int64_t a[U];                              // indices first, then values
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(jb + u, m - 1);
                const int64_t b = j < len.x ? base : base_lead;
                a[u] = JD ? m_ld<G>(off + j) + b : b + int64_t(j) * BR;
                c[set][u] = m_ld_nt<G>(reinterpret_cast<const Int2 *>(col_p + a[u]));
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[set][u] = m_ld_nt<G>(reinterpret_cast<const V2 *>(val_p + a[u]));
        };
        auto group = [&](int jb, int set) {
            T x0[U], x1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x0[u] = x(c[set][u].x);
                x1[u] = x(c[set][u].y);
            }
            if (jb + U < m) load(jb + U, set ^ 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool on = jb + u < m;
                const T s0 = __builtin_fma(v[set][u].x, x0[u], a0);
                const T s1 = __builtin_fma(v[set][u].y, x1[u], a1);
                a0 = (on && jb + u < len.x) ? s0 : a0;
                a1 = (on && jb + u < len.y) ? s1 : a1;
            }
        };
        load(0, 0);
        for (int jb = 0; jb < m; jb += 2 * U) {
            group(jb, 0);
            if (jb + U < m) group(jb + U, 1);
        }
    }
    T *y = static_cast<T *>(M.y);
    if (i < M.n_rows) m_st<G>(y + (y_perm ? i : m_ld<G>(M.perm + i)), a0);
    if (i + 1 < M.n_rows) m_st<G>(y + (y_perm ? i + 1 : m_ld<G>(M.perm + i + 1)), a1);
}

// PAIR: each wave takes two wave groups at a time (tiles hold an even number of groups, and
// every member's sort window holds whole 128-row groups).
template <class T, bool JD, int BR, bool PAIR>
__global__ __launch_bounds__(kBlock) void batch_persistent_kernel(const Member *__restrict__ members,
                                                                  const Tile *__restrict__ tiles,
                                                                  int32_t n_tiles, int32_t *counter,
                                                                  uint32_t flags) {
    const bool y_perm = flags & PJDS_Y_PERMUTED;
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(counter, 1);
        t = __shfl(t, 0);
        if (t >= n_tiles) return;                  // every wave ends here once the table is drained
        const Tile tile = tiles[t];
        const Member M = members[tile.m];
        const XGlobal<T> xa{static_cast<const T *>(M.x)};
        if (PAIR)
            for (int64_t g = tile.g0; g < tile.g1; g += 2) wave_group_pair<T, JD, BR>(M, g, y_perm, xa);
        else
            for (int64_t g = tile.g0; g < tile.g1; ++g) wave_group_pipe<T, JD, BR>(M, g, y_perm, xa);
    }
}

constexpr int kXldsThreads = 512;        // threads of a workgroup of the LDS-staged batch
constexpr int kXldsStage = 8;            // x values in flight per thread while staging
constexpr int64_t kXldsMaxBytes = 78 * 1024;   // staged x per workgroup: two workgroups fit a CU

// x staged in LDS: each workgroup pulls a tile, copies x[lo, lo + n) -- the original rows of
// the sort windows its sorted rows lie in, widened by `halo` on both sides, clipped to the
// member's columns and to `cap` values -- into LDS, and its waves then pull the tile's wave
// groups (pairs with PAIR) from a counter in LDS.  The same FMAs in the same order as
// batch_persistent_kernel; only where x is read from differs.
template <class T, bool JD, int BR, bool PAIR>
__global__ __launch_bounds__(kXldsThreads) void batch_xlds_kernel(const Member *__restrict__ members,
                                                                  const Tile *__restrict__ tiles,
                                                                  int32_t n_tiles, int32_t *counter,
                                                                  int32_t cap, int32_t halo, uint32_t flags) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    __shared__ int32_t s_tile, s_next;
    const bool y_perm = flags & PJDS_Y_PERMUTED;
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        if (threadIdx.x == 0) {
            s_tile = atomicAdd(counter, 1);
            s_next = 0;
        }
        __syncthreads();
        const int32_t t = s_tile;
        if (t >= n_tiles) return;                  // the same in every thread: the workgroup leaves together
        const Tile tile = tiles[t];
        const Member M = members[tile.m];
        const T *x = static_cast<const T *>(M.x);
        const int64_t r0 = int64_t(tile.g0) * kWave;
        const int64_t r1 = min(int64_t(tile.g1) * kWave, M.n_pad);
        const int64_t lo_r = r0 / M.window * M.window;
        const int64_t hi_r = (r1 + M.window - 1) / M.window * M.window;
        const int64_t lo = max(lo_r - int64_t(halo), int64_t(0));
        const int64_t hi = min(hi_r + int64_t(halo), M.n_cols);
        const int32_t n = int32_t(max(min(hi - lo, int64_t(cap)), int64_t(0)));
        for (int32_t k0 = 0; k0 < n; k0 += kXldsThreads * kXldsStage) {
            T v[kXldsStage];
#pragma unroll
            for (int u = 0; u < kXldsStage; ++u) {
                const int32_t k = k0 + u * kXldsThreads + int32_t(threadIdx.x);
                v[u] = k < n ? x[lo + k] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kXldsStage; ++u) {
                const int32_t k = k0 + u * kXldsThreads + int32_t(threadIdx.x);
                if (k < n) xs[k] = v[u];
            }
        }
        __syncthreads();
        const XStaged<T> xa{xs, x, uint32_t(lo), uint32_t(n)};
        for (;;) {
            int32_t u = 0;
            if (lane == 0) u = atomicAdd(&s_next, PAIR ? 2 : 1);
            u = __shfl(u, 0);
            const int64_t g = int64_t(tile.g0) + u;
            if (g >= tile.g1) break;
            if (PAIR) wave_group_pair<T, JD, BR>(M, g, y_perm, xa);
            else wave_group<T, JD, BR>(M, g, y_perm, xa);
        }
        __syncthreads();                           // LDS and s_tile are reused by the next tile
    }
}

__global__ void reset_counter_kernel(int32_t *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Persistent launch: `cap` > 0 selects the LDS-staged kernel with that many staged values.
template <class T, bool JD, int BR>
void launch_persistent(int grid, const Member *m, const Tile *t, int32_t nt, int32_t *c, uint32_t f, bool pair,
                       int32_t cap, int32_t halo, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, c);
    const size_t lds = size_t(cap) * sizeof(T);
    if (cap > 0 && pair)
        hipLaunchKernelGGL((batch_xlds_kernel<T, JD, BR, true>), dim3(grid), dim3(kXldsThreads), lds, s, m, t, nt, c, cap, halo, f);
    else if (cap > 0)
        hipLaunchKernelGGL((batch_xlds_kernel<T, JD, BR, false>), dim3(grid), dim3(kXldsThreads), lds, s, m, t, nt, c, cap, halo, f);
    else if (pair)
        hipLaunchKernelGGL((batch_persistent_kernel<T, JD, BR, true>), dim3(grid), dim3(kBlock), 0, s, m, t, nt, c, f);
    else
        hipLaunchKernelGGL((batch_persistent_kernel<T, JD, BR, false>), dim3(grid), dim3(kBlock), 0, s, m, t, nt, c, f);
}

// Allow the LDS-staged kernel its dynamic LDS beyond the default limit (gfx950 has 160 KB per CU).
template <class T, bool JD, int BR>
hipError_t allow_lds(size_t bytes, bool pair) {
    const void *k = pair ? reinterpret_cast<const void *>(&batch_xlds_kernel<T, JD, BR, true>)
                         : reinterpret_cast<const void *>(&batch_xlds_kernel<T, JD, BR, false>);
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

}  // namespace
}  // namespace pjds

using namespace pjds;

struct pjds_batch {
    int32_t mode = 0, dtype = 0, n_members = 0, n_tiles = 0;
    uint32_t flags = 0;
    bool jd = true;
    int32_t block_height = 64;
    int grid = 0;
    bool pair = false;                            // two rows per lane in the persistent kernel
    int32_t cap = 0;                              // > 0: x staged in LDS, this many values per workgroup
    int32_t halo = 0;
    std::vector<pjds_batch_member> members;       // host copies of the descriptors
    std::vector<pjds_info> infos;
    Member *d_members = nullptr;
    Tile *d_tiles = nullptr;
    int32_t *d_counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int hip_fail(hipError_t e, const char *what) {
    return fail(PJDS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void release(pjds_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_members) (void)hipFree(b->d_members);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

// Enqueue the batch's work on stream s (used directly, or under graph capture).
int enqueue(pjds_batch *b, hipStream_t s) {
    if (b->mode == PJDS_BATCH_PERSISTENT) {
        const bool jd = b->jd;
        const int br = b->block_height;
        auto go = [&](auto tag) {
            using T = decltype(tag);
            if (jd) {
                if (br == 32) launch_persistent<T, true, 32>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
                else if (br == 64) launch_persistent<T, true, 64>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
                else launch_persistent<T, true, 128>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
            } else {
                if (br == 32) launch_persistent<T, false, 32>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
                else if (br == 64) launch_persistent<T, false, 64>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
                else launch_persistent<T, false, 128>(b->grid, b->d_members, b->d_tiles, b->n_tiles, b->d_counter, b->flags, b->pair, b->cap, b->halo, s);
            }
        };
        if (b->dtype == PJDS_F64) go(double{});
        else go(float{});
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? PJDS_OK : hip_fail(e, "persistent batch launch");
    }
    for (int32_t k = 0; k < b->n_members; ++k) {
        const pjds_batch_member &m = b->members[size_t(k)];
        pjds_info info = b->infos[size_t(k)];
        info.split_len = 0;                        // rows are never split in a batch
        info.n_chunks = 0;
        int rc = pjds_spmv(&info, m.d_row_len, m.d_offsets, m.d_col_p, m.d_val_p, m.d_perm,
                           nullptr, nullptr, b->dtype, m.d_x, m.d_y, b->flags, s);
        if (rc) return rc;
    }
    return PJDS_OK;
}

}  // namespace

namespace {

// Sort window of a member in rows, as the staged kernel uses it: n_pad for a global sort.
int64_t member_window(const pjds_info &in) {
    const int64_t w = (in.flags & PJDS_LAYOUT_BLOCK) && in.sort_window < in.n_rows ? in.sort_window : in.n_pad;
    return std::max<int64_t>(w, 1);
}

// x_halo < 0: the persistent kernel gathers x through the caches; >= 0: the LDS-staged one.
int create(int32_t n_members, const pjds_batch_member *members, int32_t dtype, uint32_t flags, int32_t mode,
           int32_t groups_per_tile, int32_t x_halo, pjds_batch **out) {
    if (!out) return fail(PJDS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_members < 1 || !members) return fail(PJDS_ERR_ARG, "empty batch");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    if (flags & ~PJDS_Y_PERMUTED) return fail(PJDS_ERR_ARG, "unsupported batch flags 0x%x", flags);
    if (mode != PJDS_BATCH_PERSISTENT && mode != PJDS_BATCH_GRAPH && mode != PJDS_BATCH_DIRECT)
        return fail(PJDS_ERR_ARG, "mode %d", mode);
    const bool staged = x_halo >= 0;
    const pjds_info &first = *members[0].info;
    for (int32_t k = 0; k < n_members; ++k) {
        const pjds_batch_member &m = members[k];
        if (!m.info) return fail(PJDS_ERR_ARG, "member %d: info is NULL", k);
        const pjds_info &in = *m.info;
        if (in.block_height != first.block_height || (in.flags & PJDS_LAYOUT_BLOCK) != (first.flags & PJDS_LAYOUT_BLOCK))
            return fail(PJDS_ERR_ARG, "member %d: every member needs the same block height and layout", k);
        if (in.flags & PJDS_LANES_MASK)
            return fail(PJDS_ERR_UNSUPPORTED, "member %d: a matrix with several lanes per row cannot join a batch", k);
        if (in.block_height != 32 && in.block_height != 64 && in.block_height != 128)
            return fail(PJDS_ERR_ARG, "member %d: block_height %d", k, in.block_height);
        if (in.n_rows < 0 || in.n_pad < in.n_rows || in.n_pad % in.block_height)
            return fail(PJDS_ERR_ARG, "member %d: inconsistent info", k);
        if (in.n_rows && (!m.d_row_len || !m.d_offsets || !m.d_y))
            return fail(PJDS_ERR_ARG, "member %d: NULL device array", k);
        if (in.nnz_stored && (!m.d_col_p || !m.d_val_p || !m.d_x))
            return fail(PJDS_ERR_ARG, "member %d: NULL device array", k);
        // the staged kernel copies each tile's range of x into LDS, even without entries
        if (staged && in.n_rows && in.n_cols && !m.d_x) return fail(PJDS_ERR_ARG, "member %d: d_x is NULL", k);
        if (in.n_rows && !(flags & PJDS_Y_PERMUTED) && !m.d_perm)
            return fail(PJDS_ERR_ARG, "member %d: d_perm is NULL (needed to scatter y)", k);
        if (ceil_div(in.n_pad, kWave) > INT32_MAX) return fail(PJDS_ERR_OVERFLOW, "member %d too large", k);
    }
    pjds_batch *b = new (std::nothrow) pjds_batch;
    if (!b) return fail(PJDS_ERR_NOMEM, "host allocation failed");
    b->mode = mode;
    b->dtype = dtype;
    b->flags = flags;
    b->n_members = n_members;
    b->jd = !(first.flags & PJDS_LAYOUT_BLOCK);
    b->block_height = first.block_height;
    b->members.assign(members, members + n_members);
    for (int32_t k = 0; k < n_members; ++k) b->infos.push_back(*members[k].info);

    if (mode == PJDS_BATCH_PERSISTENT) {
        // two rows per lane when every tile holds an even number of wave groups and every
        // member is sorted in windows of whole 128-row groups (block layout).  With a global
        // sort the rows of a wave come from all over the matrix and the doubled gathers per
        // lane cost more than the wider loads save (measured 7% slower), so it keeps one row.
        bool windowed = true;
        for (int32_t k = 0; k < n_members; ++k) {
            const pjds_info &in = *members[k].info;
            if (!(in.flags & PJDS_LAYOUT_BLOCK) || in.sort_window >= in.n_rows || in.sort_window % 128) windowed = false;
        }
        // default tiles: 8 wave groups; with x staged, 32 for windowed members (a workgroup's
        // waves then share each tile's copy of x; 2% faster than 16) and 8 otherwise (4%
        // faster than 16 for globally sorted members, whose staged range is the whole member)
        if (groups_per_tile <= 0) groups_per_tile = staged && windowed ? 32 : 8;
        b->pair = windowed && groups_per_tile % 2 == 0;
        std::vector<Member> dm(static_cast<size_t>(n_members));
        // Members are visited largest first and each member's tiles stay together, so the
        // waves running at any moment share one member's x in cache; the small members at
        // the end fill the tail of the launch.
        std::vector<int32_t> order(static_cast<size_t>(n_members));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
            return members[a].info->nnz_stored > members[c].info->nnz_stored;
        });
        std::vector<Tile> sorted;
        for (int32_t k = 0; k < n_members; ++k) {
            const pjds_batch_member &m = members[k];
            const pjds_info &in = *m.info;
            dm[size_t(k)] = Member{m.d_row_len, m.d_offsets, m.d_col_p, m.d_val_p, m.d_perm, m.d_x, m.d_y,
                                   in.n_rows, in.n_pad, in.n_cols, member_window(in)};
        }
        // the largest x range a tile of the staged kernel needs (the kernel's own formula)
        const int64_t esz = dtype == PJDS_F64 ? 8 : 4;
        int64_t need = 0;
        for (int32_t k : order) {
            const pjds_info &in = *members[k].info;
            const int64_t groups = ceil_div(in.n_pad, kWave), w = member_window(in);
            for (int64_t g = 0; g < groups; g += groups_per_tile) {
                const int64_t g1 = std::min(groups, g + groups_per_tile);
                sorted.push_back(Tile{k, int32_t(g), int32_t(g1), 0});
                if (staged) {
                    const int64_t lo = std::max<int64_t>(g * kWave / w * w - x_halo, 0);
                    const int64_t hi = std::min<int64_t>(ceil_div(std::min(g1 * kWave, in.n_pad), w) * w + x_halo, in.n_cols);
                    need = std::max(need, hi - lo);
                }
            }
        }
        if (sorted.size() > size_t(INT32_MAX)) { release(b); return fail(PJDS_ERR_OVERFLOW, "too many tiles"); }
        b->n_tiles = int32_t(sorted.size());
        int dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) { release(b); return hip_fail(e, "device query"); }
        if (staged) {
            // wider ranges are cut at the cap (their far ends are read from global memory)
            b->cap = int32_t(std::max<int64_t>(std::min(need, kXldsMaxBytes / esz), 1));
            b->halo = x_halo;
            const int64_t bytes = int64_t(b->cap) * esz;
            const int per_cu = int(std::max<int64_t>(1, std::min<int64_t>(4, (160 * 1024) / (bytes + 1024))));
            b->grid = std::max(1, cus) * per_cu;
            auto allow = [&](auto tag) -> hipError_t {
                using T = decltype(tag);
                const int br = b->block_height;
                if (b->jd) return br == 32 ? allow_lds<T, true, 32>(size_t(bytes), b->pair)
                                 : br == 64 ? allow_lds<T, true, 64>(size_t(bytes), b->pair)
                                            : allow_lds<T, true, 128>(size_t(bytes), b->pair);
                return br == 32 ? allow_lds<T, false, 32>(size_t(bytes), b->pair)
                     : br == 64 ? allow_lds<T, false, 64>(size_t(bytes), b->pair)
                                : allow_lds<T, false, 128>(size_t(bytes), b->pair);
            };
            e = dtype == PJDS_F64 ? allow(double{}) : allow(float{});
            if (e != hipSuccess) { release(b); return hip_fail(e, "LDS size of the staged batch kernel"); }
        } else {
            b->grid = std::max(1, cus) * 8;        // 8 workgroups (32 waves) per CU
        }
        e = hipMalloc(&b->d_members, sizeof(Member) * dm.size());
        if (e == hipSuccess) e = hipMalloc(&b->d_tiles, sizeof(Tile) * std::max<size_t>(sorted.size(), 1));
        if (e == hipSuccess) e = hipMalloc(&b->d_counter, 256);
        if (e == hipSuccess) e = hipMemcpy(b->d_members, dm.data(), sizeof(Member) * dm.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !sorted.empty()) e = hipMemcpy(b->d_tiles, sorted.data(), sizeof(Tile) * sorted.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) { release(b); return hip_fail(e, "batch tables"); }
    }
    if (mode != PJDS_BATCH_DIRECT) {
        // capture on a private stream (the default stream cannot be captured)
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) { release(b); return hip_fail(e, "capture stream"); }
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? enqueue(b, cs) : hip_fail(e, "begin capture");
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        b->graph = g;
        if (rc == PJDS_OK && e2 != hipSuccess) rc = hip_fail(e2, "end capture");
        if (rc == PJDS_OK) {
            e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "graph instantiate");
        }
        (void)hipStreamDestroy(cs);
        if (rc) { release(b); return rc; }
    }
    *out = b;
    return PJDS_OK;
}

}  // namespace

extern "C" {

int pjds_batch_create(int32_t n_members, const pjds_batch_member *members, int32_t dtype,
                      uint32_t flags, int32_t mode, int32_t groups_per_tile, pjds_batch **out) {
    return create(n_members, members, dtype, flags, mode, groups_per_tile, -1, out);
}

int pjds_batch_create_xlds(int32_t n_members, const pjds_batch_member *members, int32_t dtype,
                           uint32_t flags, int32_t groups_per_tile, int32_t x_halo, pjds_batch **out) {
    if (x_halo < 0) {
        if (out) *out = nullptr;
        return fail(PJDS_ERR_ARG, "x_halo %d", x_halo);
    }
    return create(n_members, members, dtype, flags, PJDS_BATCH_PERSISTENT, groups_per_tile, x_halo, out);
}

int pjds_batch_launch(pjds_batch *b, void *stream) {
    if (!b) return fail(PJDS_ERR_ARG, "batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->mode == PJDS_BATCH_DIRECT) return enqueue(b, s);
    hipError_t e = hipGraphLaunch(b->exec, s);
    return e == hipSuccess ? PJDS_OK : hip_fail(e, "graph launch");
}

int pjds_batch_info(const pjds_batch *b, int32_t *n_tiles, int32_t *grid) {
    if (!b) return fail(PJDS_ERR_ARG, "batch is NULL");
    if (n_tiles) *n_tiles = b->n_tiles;
    if (grid) *grid = b->grid;
    return PJDS_OK;
}

int pjds_batch_destroy(pjds_batch *b) {
    release(b);
    return PJDS_OK;
}

}  // extern "C"
