// Sparse matrix-vector kernels for MI355X (gfx950): pJDS (Listing 2 of Kreutzer et al.,
// arXiv:1112.5588), ELLPACK-R (Listing 1), CSR, and the many-right-hand-side pJDS product.
//
// Mapping.  One lane owns one (sorted) row; one 64-lane wavefront owns 64 consecutive rows
// (a "wave group").  With the block height b_r = 64 a wave group is exactly one pJDS block,
// so every lane of a wave loops to the same block maximum M_b and the stored column
// segment of that block (64 values, 64 indices) is one coalesced 512 B + 256 B access per
// step.  b_r = 32 puts two blocks in a wave, b_r = 128 spreads a block over two waves; the
// loop bound is always the wave's own longest row, and each lane masks its arithmetic with
// its own row length, so padding never enters a sum.  Rows are sorted longest first inside
// windows that hold whole waves, so lane 0 holds the wave's longest row: its length is the
// loop bound, and a lane past the end of its own row re-reads lane 0's slot instead of its
// own padding slot.  That address and the x element it points to are already being fetched
// for lane 0, so padding costs neither HBM traffic nor extra cache lines.
//
// Streams.  Values and column indices are read exactly once per product, so they are
// loaded non-temporally; x goes through the normal cached path (it is re-read by every
// row that references it).  With PJDS_XCD_REMAP workgroups are renumbered so that each XCD
// (8 per MI355X, each with its own L2) processes one contiguous range of row blocks.
//
// Long rows.  Wave groups whose longest row exceeds split_len are cut into work items of
// split_len steps, scheduled first.  Each item writes its 64 partial sums to the workspace;
// the item that completes a group last (device-scope counter) adds the partials in item
// order and stores y, then resets the counter.  The order of additions is therefore fixed
// and results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "device.h"
#include "launch.h"

namespace pjds {
namespace {

constexpr int kBlock = 256;               // threads per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
#ifndef PJDS_UNROLL
#define PJDS_UNROLL 8
#endif
constexpr int kUnroll = PJDS_UNROLL;      // independent entries in flight per lane
constexpr int kStage = 8;                 // x values in flight per thread while staging into LDS

__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t grid) {
    // Hardware hands workgroup b to XCD b % 8; give XCD x the contiguous logical range
    // [x*q + min(x, r), ...) of length q + (x < r).  A bijection on [0, grid).
    const uint32_t x = b % kXcds, k = b / kXcds, q = grid / kXcds, r = grid % kXcds;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ uint32_t logical_block(uint32_t flags) {
    return (flags & PJDS_XCD_REMAP) ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
}

// Tiles of the LDS product: contiguous ranges per XCD with PJDS_XCD_REMAP, else runs of
// kXcdGroup tiles per XCD.
__device__ __forceinline__ uint32_t tile_block(uint32_t flags) {
    return (flags & PJDS_XCD_REMAP) ? xcd_remap(blockIdx.x, gridDim.x) : xcd_group(blockIdx.x, gridDim.x);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

// Lowest lane of the wave whose row is the longest (len == m, m > 0); for unsorted rows.
__device__ __forceinline__ int lead_lane(int len, int m) {
    return __builtin_ctzll(__ballot(len == m));
}

// Where entry j of a row lives, given the row's base position b (see each format).
template <bool JD, int BR>
struct PjdsAddr {                       // JD: col_start[j] + i;  block: block_start + j*BR + r
    const int64_t *off;
    __device__ int64_t base(int64_t i) const { return JD ? i : off[i / BR] + (i % BR); }
    __device__ int64_t operator()(int j, int64_t b) const { return JD ? off[j] + b : b + int64_t(j) * BR; }
};
struct EllrAddr {                       // ELLPACK-R: j * n_pad + i
    int64_t n_pad;
    __device__ int64_t base(int64_t i) const { return i; }
    __device__ int64_t operator()(int j, int64_t b) const { return int64_t(j) * n_pad + b; }
};

// Reads of the right-hand side: x[c * ld + off] through the caches ...
template <class T>
struct XGlobal {
    const T *__restrict__ x;
    int64_t ld, off;
    __device__ T operator()(int32_t c) const { return x[int64_t(c) * ld + off]; }
};
// ... or, for columns inside the window [lo, lo + n) staged in LDS, from LDS.
template <class T>
struct XStaged {
    const T *__restrict__ x;
    const T *lds;
    int64_t lo;
    uint32_t n;
    __device__ T operator()(int32_t c) const {
        return staged_or_global<T>(lds, uint32_t(int64_t(c) - lo), n, 1, x, c);
    }
    // Two phases for a group of reads: every LDS read first, then the global reads of the
    // columns outside the staged range.  A global read writes the register of its LDS read
    // and must wait for it to land; issued after all of them, only the first such wait costs.
    template <int K>
    __device__ __forceinline__ void group(T (&v)[K], const int32_t (&c)[K]) const {
        typedef __attribute__((address_space(3))) const T LdsT;
        bool out[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t d = uint32_t(int64_t(c[k]) - lo);
            out[k] = d >= n;
            v[k] = ((const LdsT *)lds)[out[k] ? 0u : d];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (out[k]) v[k] = x[c[k]];
    }
};

// Reads of a group through the caches (XGlobal): one gather per entry.
template <class T, int K>
__device__ __forceinline__ void gather_group(const XGlobal<T> &xr, T (&v)[K], const int32_t (&c)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = xr(c[k]);
}
template <class T, int K>
__device__ __forceinline__ void gather_group(const XStaged<T> &xr, T (&v)[K], const int32_t (&c)[K]) {
    xr.group(v, c);
}

// What a product writes: y[r] = alpha * (A x)[r] + b * z[r], with b = beta, or b = bscale *
// (*beta_dev) when the coefficient lives in device memory (an iterative solver's scalar that
// the host never reads).  z is indexed like y and may be y itself.  Plain product: alpha = 1,
// z = nullptr (then y = A x exactly).
template <class T>
struct Epilogue {
    T alpha, beta;
    const T *z;
    const T *beta_dev;
    T bscale;
    const T *alpha_dev;                 // if set, alpha = *alpha_dev
    double *dot;                        // if set, per-workgroup sums of y_i * x_i (staged products)
    const double *norm_part;            // if set, a Lanczos step's scalars come from these
    int32_t n_norm;                     // partial sums (EpiArgs)
    const double *inv_prev;
    double *inv_out;
    double *beta_out;
    __device__ T operator()(T acc, int64_t r) const {
        const T a = alpha_dev ? alpha_dev[0] : alpha;
        if (!z) return a * acc;
        const T b = beta_dev ? bscale * beta_dev[0] : beta;
        return __builtin_fma(b, z[r], a * acc);
    }
    // y[r] = (*this)(acc, r).  The plain product's y is written once and not read back by the
    // kernel, so it is stored non-temporally (keeps the caches for x); a solver's update, whose
    // result the next kernel reads at once, is stored normally.
    __device__ void store(T *y, int64_t r, T acc) const { put(y, r, (*this)(acc, r)); }
    __device__ void put(T *y, int64_t r, T v) const {
        if (!z && !alpha_dev) __builtin_nontemporal_store(v, y + r);
        else y[r] = v;
    }
};

// U consecutive entries j in [jb, jb+U) added into acc: U independent value/index loads,
// then U gathers, then U FMAs.  A lane past the end of its row reads the lead row's slot (an
// entry that exists for every j below the wave's longest row) and keeps acc.  With CLAMP,
// steps at or past j1 re-read step j1 - 1 and are masked, so a ragged tail of any length
// costs one round trip to memory without a load past j1.
template <int U, bool CLAMP, class T, class Addr, class XR>
__device__ __forceinline__ void row_steps(T &acc, int jb, int j1, int len, int64_t base, int64_t base_lead,
                                          const Addr &addr, const int32_t *__restrict__ col_p,
                                          const T *__restrict__ val_p, const XR &xr) {
    T v[U];
    int32_t c[U];
    int64_t a[U];                                      // indices first, then values
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = CLAMP ? min(jb + u, j1 - 1) : jb + u;
        a[u] = addr(j, j < len ? base : base_lead);
        c[u] = ld_stream(col_p + a[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld_stream(val_p + a[u]);
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = xr(c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const T s = __builtin_fma(v[u], xv[u], acc);
        acc = (jb + u < len && (!CLAMP || jb + u < j1)) ? s : acc;
    }
}

// Sum of the calling lane's row entries j in [j0, j1) (Listing 1 / Listing 2 inner loop).
// base is the lane's own first slot, base_lead that of the wave's longest row; j1 is
// wave-uniform and <= that row's length.  Full groups of kUnroll steps, then one clamped
// group for the remainder (8, 4 or 2 wide; a single step exactly).
template <class T, class Addr, class XR>
__device__ __forceinline__ T row_range_sum(int64_t base, int64_t base_lead, int len, int j0, int j1,
                                           const Addr &addr, const int32_t *__restrict__ col_p,
                                           const T *__restrict__ val_p, const XR &xr) {
    T acc = T(0);
    int jb = j0;
    for (; jb + kUnroll <= j1; jb += kUnroll)
        row_steps<kUnroll, false>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    const int r = j1 - jb;
    if (kUnroll > 8 && r > 8) row_steps<kUnroll, true>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    else if (r > 4) row_steps<8, true>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    else if (r > 2) row_steps<4, true>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    else if (r == 2) row_steps<2, false>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    else if (r == 1) row_steps<1, false>(acc, jb, j1, len, base, base_lead, addr, col_p, val_p, xr);
    return acc;
}

// R adjacent sorted rows per lane (R = kRowsPerLane).  At step j the slots of rows i .. i+R-1
// (i a multiple of R) are neighbours in both layouts, so a lane reads their values with one
// R-wide load and their column indices with another: a wave instruction moves R times the
// bytes of a 1-wide load.  Row i is the lane's longest (rows are sorted), so a lane past row i
// re-reads lane 0's slots, and padding slots of its shorter rows are read but never added.
constexpr int kRowsPerLane = 2;
template <class T, int R>
struct VecR { typedef T type __attribute__((ext_vector_type(R))); };
template <int R>
struct IdxR { typedef int32_t type __attribute__((ext_vector_type(R))); };

// R rows per lane with the next group of steps loading while the current one gathers: the
// values and indices of steps [jb + U, jb + 2U) are issued after the gathers of steps
// [jb, jb + U) and before their FMAs, so a wave keeps a group of matrix loads in flight while
// it waits for x.  The loop body is one block with a fixed number of loads behind the
// gathers, so the FMAs wait for the gathers only.  Every group is U steps wide; steps at or
// past the wave's longest row m re-read step m - 1 (lines already fetched) and are masked,
// so no load reaches past the longest row.  One FMA per entry in stored order per row, as in
// row_steps.  The caller loads the first group (steps [0, U)) into ga, so it can issue those
// loads early, before work that does not depend on them.
template <int U, int R, class T>
struct StepGroup {
    typedef typename VecR<T, R>::type V;
    typedef typename IdxR<R>::type I;
    V v[U];
    I c[U];
    template <class Addr>
    __device__ __forceinline__ void load(int jb, int m, int len0, int64_t base, int64_t base_lead, const Addr &addr,
                                         const int32_t *__restrict__ col_p, const T *__restrict__ val_p) {
        // the indices first: the gathers wait for them only, the values can still be in flight
        int64_t a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(jb + u, m - 1);
            a[u] = addr(j, j < len0 ? base : base_lead);
            c[u] = __builtin_nontemporal_load(reinterpret_cast<const I *>(col_p + a[u]));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(reinterpret_cast<const V *>(val_p + a[u]));
    }
    template <class XR>
    __device__ __forceinline__ void gather(T (&xv)[U * R], const XR &xr) const {
        int32_t cc[U * R];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < R; ++q) cc[u * R + q] = c[u][q];
        gather_group(xr, xv, cc);
    }
    __device__ __forceinline__ void fma(T (&acc)[R], const T (&xv)[U * R], int jb, const int (&len)[R]) const {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const T s = __builtin_fma(v[u][q], xv[u * R + q], acc[q]);
                acc[q] = jb + u < len[q] ? s : acc[q];
            }
    }
};

template <int R, class T, class Addr, class XR>
__device__ __forceinline__ void row_group_sum_pipe(T (&acc)[R], StepGroup<(R >= 4 ? 2 : 4), R, T> &ga, int64_t base, int64_t base_lead, const int (&len)[R],
                                                   int m, const Addr &addr, const int32_t *__restrict__ col_p,
                                                   const T *__restrict__ val_p, const XR &xr) {
    constexpr int U = R >= 4 ? 2 : 4;
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = T(0);
    if (m <= 0) return;
    // two register sets in turn, so the loads in flight never have to land for a copy
    StepGroup<U, R, T> gb;
    auto step = [&](const StepGroup<U, R, T> &cur, StepGroup<U, R, T> &nxt, int jb) {
        T xv[U * R];
        cur.gather(xv, xr);
        nxt.load(jb + U, m, len[0], base, base_lead, addr, col_p, val_p);
        __builtin_amdgcn_sched_barrier(0);      // keep every next-group load ahead of the FMAs
        cur.fma(acc, xv, jb, len);
    };
    auto last = [&](const StepGroup<U, R, T> &cur, int jb) {
        T xv[U * R];
        cur.gather(xv, xr);
        cur.fma(acc, xv, jb, len);
    };
    const int groups = (m + U - 1) / U;
    int k = 1, jb = 0;
    for (; k + 1 < groups; k += 2, jb += 2 * U) {
        step(ga, gb, jb);
        step(gb, ga, jb + U);
    }
    if (k < groups) {
        step(ga, gb, jb);
        last(gb, jb + U);
    } else {
        last(ga, jb);
    }
}

template <class T, bool JD, int BR>
__global__ __launch_bounds__(kBlock) void pjds_spmv_kernel(
    int64_t n_rows, int64_t n_pad, int64_t n_groups, int64_t n_chunks, int32_t split_len,
    const int32_t *__restrict__ row_len, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ col_p, const T *__restrict__ val_p,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ sched,
    T *__restrict__ partials, int32_t *__restrict__ counters,
    const T *__restrict__ x, T *y, Epilogue<T> epi, uint32_t flags) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = int64_t(logical_block(flags)) * kWavesPerBlock + (threadIdx.x >> 6);
    const bool y_perm = flags & PJDS_Y_PERMUTED;

    if (w < n_chunks) {
        // ---- one work item of a long wave group
        const int32_t g = sched[4 * w + 0], c = sched[4 * w + 1], nc = sched[4 * w + 2], first = sched[4 * w + 3];
        const int64_t i = int64_t(g) * kWave + lane;
        const PjdsAddr<JD, BR> addr{offsets};
        int len = row_len[i < n_pad ? i : n_pad - 1];      // clamped, then masked (see below)
        const int64_t base = addr.base(i);
        if (i >= n_pad) len = 0;
        const int m = wave_first(len);
        const int j0 = c * split_len, j1 = min(j0 + split_len, m);
        const T part = row_range_sum(base, wave_first(base), len, j0, j1, addr, col_p, val_p, XGlobal<T>{x, 1, 0});
        partials[w * kWave + lane] = part;
        __threadfence();                                    // publish the partial sums
        int last = 0;
        if (lane == 0) last = atomicAdd(&counters[first], 1) == nc - 1;
        last = __shfl(last, 0);
        if (last) {
            __threadfence();                                // see every item's partials
            const volatile T *pp = partials + int64_t(first) * kWave + lane;
            T s = pp[0];
            for (int q = 1; q < nc; ++q) s += pp[int64_t(q) * kWave];
            if (i < n_rows) {
                const int64_t r = y_perm ? i : perm[i];
                epi.store(y, r, s);
            }
            if (lane == 0) counters[first] = 0;             // ready for the next product
        }
        return;
    }
    const int64_t g = w - n_chunks;
    if (g >= n_groups) return;
    const int64_t i = g * kWave + lane;
    const PjdsAddr<JD, BR> addr{offsets};
    // the length loads at an index clamped into range and is masked afterwards, and no early
    // exit sits between it and the offset load: both are in flight together (a load in a
    // branch, or one the compiler may sink below a branch, costs a round trip of its own)
    int len = row_len[i < n_pad ? i : n_pad - 1];
    const int64_t base = addr.base(i);
    if (i >= n_pad) len = 0;
    const int m = wave_first(len);
    const bool by_items = split_len > 0 && m > split_len;  // done by the work items above
    const T acc = row_range_sum(base, wave_first(base), len, 0, by_items ? 0 : m, addr, col_p, val_p,
                                XGlobal<T>{x, 1, 0});
    if (!by_items && i < n_rows) {
        const int64_t r = y_perm ? i : perm[i];
        epi.store(y, r, acc);
    }
}

// The plain product with kRowsPerLane adjacent rows per lane (PJDS_TWO_ROWS): one wave per
// 64 R consecutive sorted rows, x through the caches.  For matrices without long-row work
// items whose sort holds whole 64 R-row groups (a global sort, or windows that are a multiple
// of 64 R); same FMAs in the same order per row as pjds_spmv_kernel.
template <class T, bool JD, int BR>
__global__ __launch_bounds__(kBlock) void pjds_spmv2_kernel(
    int64_t n_rows, int64_t n_pad, int64_t n_waves, const int32_t *__restrict__ row_len,
    const int64_t *__restrict__ offsets, const int32_t *__restrict__ col_p, const T *__restrict__ val_p,
    const int32_t *__restrict__ perm, const T *__restrict__ x, T *y, Epilogue<T> epi, uint32_t flags) {
    constexpr int R = kRowsPerLane;
    typedef typename IdxR<R>::type I;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = int64_t(logical_block(flags)) * kWavesPerBlock + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    const int64_t i = w * (kWave * R) + int64_t(R) * lane;
    I lv = *reinterpret_cast<const I *>(row_len + (i < n_pad ? i : n_pad - R));   // clamped, then masked
    if (i >= n_pad) lv = I{};
    const PjdsAddr<JD, BR> addr{offsets};
    const int64_t base = addr.base(i < n_pad ? i : n_pad - R);    // n_pad is a multiple of R
    int len[R];
#pragma unroll
    for (int q = 0; q < R; ++q) len[q] = lv[q];
    const int m = wave_first(len[0]);
    T acc[R];
    StepGroup<(R >= 4 ? 2 : 4), R, T> g0;      // first group of steps, then two sets in turn
    const int64_t bl = wave_first(base);
    if (m > 0) g0.load(0, m, len[0], base, bl, addr, col_p, val_p);
    row_group_sum_pipe<R>(acc, g0, base, bl, len, m, addr, col_p, val_p, XGlobal<T>{x, 1, 0});
    const bool y_perm = flags & PJDS_Y_PERMUTED;
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (i + q < n_rows) {
            const int64_t r = y_perm ? i + q : perm[i + q];
            epi.store(y, r, acc[q]);
        }
}

// Row lengths as the staged products read them: int32 (the converted rowmax array), or one
// byte each (L8, PJDS_ROW_LEN8; the pointer then addresses uint8_t lengths).
template <bool L8>
__device__ __forceinline__ int row_len_at(const int32_t *rl, int64_t i) {
    if (L8) return reinterpret_cast<const uint8_t *>(rl)[i];
    return rl[i];
}
// The lengths of rows i and i + 1 (i even): one 8-byte or one 2-byte load.
template <bool L8>
__device__ __forceinline__ typename IdxR<2>::type row_len_pair(const int32_t *rl, int64_t i) {
    typedef typename IdxR<2>::type I;
    if (!L8) return *reinterpret_cast<const I *>(rl + i);
    const uint16_t p = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(rl) + i);
    I r;
    r[0] = p & 0xff;
    r[1] = p >> 8;
    return r;
}

// pJDS product with the right-hand side staged in LDS (block layout with a sort window).
// A workgroup of NT threads (256 or 512) owns `tile` consecutive sorted rows (a multiple of
// 256; NT = 512 when the tile is a multiple of 512, so a 512-row tile runs in one pass).
// Sorting never moves a row out of its window of `window` original rows, so the tile's rows
// are original rows inside [lo_r, hi_r), the union of the windows the tile touches.  The workgroup copies x[lo_r - halo, hi_r + halo) (clipped to the matrix) into
// LDS once with coalesced loads, then runs its rows NT at a time; entries whose column falls
// in the staged range read x from LDS, the others from global memory.  Rows are never split
// here.  Same arithmetic order as pjds_spmv_kernel.
template <class T, int BR, int NT, bool L8>
__global__ __launch_bounds__(NT) void pjds_spmv_lds_kernel(
    int64_t n_rows, int64_t n_cols, int64_t n_pad, int64_t window, int64_t halo, int64_t tile,
    const int32_t *__restrict__ row_len, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ col_p, const T *__restrict__ val_p,
    const int32_t *__restrict__ perm, const T *__restrict__ x, T *y, Epilogue<T> epi, uint32_t flags) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    const int64_t r0 = int64_t(tile_block(flags)) * tile;            // first sorted row of the tile
    const int64_t lo_r = r0 / window * window;
    const int64_t hi_r = (r0 + tile + window - 1) / window * window;
    const int64_t lo = lo_r - halo > 0 ? lo_r - halo : 0;
    const int64_t hi = hi_r + halo < n_cols ? hi_r + halo : n_cols;
    // The first rows' lengths and block offsets go out before the copy of x, so their latency
    // overlaps it (the barrier waits for LDS traffic only).  Rows past n_pad (length 0)
    // address the last real row, so the offsets are never read out of range.
    const PjdsAddr<false, BR> addr{offsets};
    int64_t i = r0 + threadIdx.x;
    int len = row_len_at<L8>(row_len, i < n_pad ? i : n_pad - 1);     // clamped, then masked
    int64_t base = addr.base(i < n_pad ? i : n_pad - 1);
    if (i >= n_pad) len = 0;
    // copy x[lo, hi) with kStage independent loads in flight per thread
    for (int64_t c0 = lo + threadIdx.x; c0 < hi; c0 += int64_t(NT) * kStage) {
        T v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int64_t c = c0 + int64_t(u) * NT;
            v[u] = c < hi ? x[c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int64_t c = c0 + int64_t(u) * NT;
            if (c < hi) xs[c - lo] = v[u];
        }
    }
    __syncthreads();
    const XStaged<T> xr{x, xs, lo, uint32_t(hi > lo ? hi - lo : 0)};
    const bool y_perm = flags & PJDS_Y_PERMUTED;
    for (int64_t rb = r0;;) {
        const int m = wave_first(len);
        const T acc = row_range_sum(base, wave_first(base), len, 0, m, addr, col_p, val_p, xr);
        if (i < n_rows) {
            const int64_t r = y_perm ? i : perm[i];
            epi.store(y, r, acc);
        }
        rb += NT;
        if (rb >= r0 + tile || rb >= n_pad) break;
        i = rb + threadIdx.x;
        len = row_len_at<L8>(row_len, i < n_pad ? i : n_pad - 1);
        base = addr.base(i < n_pad ? i : n_pad - 1);
        if (i >= n_pad) len = 0;
    }
}

// The LDS-staged product with kRowsPerLane adjacent rows per lane (PJDS_TWO_ROWS): NT
// threads run R NT rows per pass; a wave covers 64 R sorted rows, so the sort window must
// hold whole groups of that size (their longest row is lane 0's first).  Same staging as
// above; each row's sum is the same FMAs in the same order as pjds_spmv_kernel.
template <class T, int BR, int NT, bool L8>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void pjds_spmv_lds2_kernel(
    int64_t n_rows, int64_t n_cols, int64_t n_pad, int64_t window, int64_t halo, int64_t tile,
    const int32_t *__restrict__ row_len, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ col_p, const T *__restrict__ val_p,
    const int32_t *__restrict__ perm, const T *__restrict__ x, T *y, Epilogue<T> epi, uint32_t flags) {
    constexpr int R = kRowsPerLane;
    typedef typename IdxR<R>::type I;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    const int64_t r0 = int64_t(tile_block(flags)) * tile;
    const int64_t lo_r = r0 / window * window;
    const int64_t hi_r = (r0 + tile + window - 1) / window * window;
    const int64_t lo = lo_r - halo > 0 ? lo_r - halo : 0;
    const int64_t hi = hi_r + halo < n_cols ? hi_r + halo : n_cols;
    const PjdsAddr<false, BR> addr{offsets};
    // n_pad is a multiple of R, so a group never straddles it; groups past it address the
    // last real group
    int64_t i = r0 + R * int64_t(threadIdx.x);
    // the lengths load at an index clamped into range and are masked afterwards: a load in a
    // branch would have to land (and be unpacked) inside it, before anything else is issued
    I lv = row_len_pair<L8>(row_len, i < n_pad ? i : n_pad - R);
    int64_t base = addr.base(i < n_pad ? i : n_pad - R);
    if (i >= n_pad) lv = I{};
    // a Lanczos step: this thread's share of the previous pass's partial sums, loaded with the
    // copy of x and added up after it
    double npart = 0.0;
    if (epi.norm_part) {
        npart = int(threadIdx.x) < epi.n_norm ? epi.norm_part[threadIdx.x] : 0.0;   // no wait here
        for (int q = threadIdx.x + NT; q < epi.n_norm; q += NT) npart += epi.norm_part[q];
    }
    // the first chunk of x to stage, then the first group of matrix steps of the first pass
    // (it needs only the lengths and offsets), then the copy into LDS: those matrix loads are
    // in flight across the copy and the barrier
    T sv[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int64_t c = lo + threadIdx.x + int64_t(u) * NT;
        sv[u] = c < hi ? x[c] : T(0);
    }
    StepGroup<(R >= 4 ? 2 : 4), R, T> g0;
    int len0[R];
#pragma unroll
    for (int q = 0; q < R; ++q) len0[q] = lv[q];
    const int m0 = wave_first(len0[0]);
    const int64_t bl0 = wave_first(base);
    if (m0 > 0) g0.load(0, m0, len0[0], base, bl0, addr, col_p, val_p);
    __builtin_amdgcn_sched_barrier(0);      // keep those loads ahead of the LDS writes
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int64_t c = lo + threadIdx.x + int64_t(u) * NT;
        if (c < hi) xs[c - lo] = sv[u];
    }
    for (int64_t c0 = lo + threadIdx.x + int64_t(NT) * kStage; c0 < hi; c0 += int64_t(NT) * kStage) {
        T v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int64_t c = c0 + int64_t(u) * NT;
            v[u] = c < hi ? x[c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int64_t c = c0 + int64_t(u) * NT;
            if (c < hi) xs[c - lo] = v[u];
        }
    }
    __shared__ double wsum[NT / kWave];
    Epilogue<T> ep = epi;
    if (epi.norm_part) {
        // the same fixed-order sum in every workgroup: butterfly inside each wave, then the
        // waves in order; b = sqrt(sum) is beta_j (the norm of the Lanczos vector u_j)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) npart += __shfl_xor(npart, off);
        if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = npart;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < NT / kWave; ++w) t += wsum[w];
        const double b = sqrt(t), inv = 1.0 / b;
        ep.alpha = T(inv);
        ep.alpha_dev = nullptr;
        if (epi.z) {
            ep.beta = T(-(b * epi.inv_prev[0]));
            ep.beta_dev = nullptr;
        }
        if (r0 == 0 && threadIdx.x == 0) {
            epi.inv_out[0] = inv;
            if (epi.beta_out) epi.beta_out[0] = b;
        }
    }
    __syncthreads();                    // x staged; wsum free again
    const XStaged<T> xr{x, xs, lo, uint32_t(hi > lo ? hi - lo : 0)};
    const bool y_perm = flags & PJDS_Y_PERMUTED;
    double dsum = 0.0;                  // this thread's rows' y_i * x_i (epi.dot only)
    for (int64_t rb = r0;;) {
        int len[R];
#pragma unroll
        for (int q = 0; q < R; ++q) len[q] = lv[q];
        T acc[R];
        if (rb == r0) {
            row_group_sum_pipe<R>(acc, g0, base, bl0, len0, m0, addr, col_p, val_p, xr);
        } else {
            const int m = wave_first(len[0]);
            const int64_t bl = wave_first(base);
            if (m > 0) g0.load(0, m, len[0], base, bl, addr, col_p, val_p);
            row_group_sum_pipe<R>(acc, g0, base, bl, len, m, addr, col_p, val_p, xr);
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (i + q < n_rows) {
                const int64_t r = y_perm ? i + q : perm[i + q];
                const T v = ep(acc[q], r);
                ep.put(y, r, v);
                // a square matrix in the permuted basis: row i's own entry of x is staged
                if (epi.dot) dsum = __builtin_fma(double(v), double(xs[i + q - lo]), dsum);
            }
        rb += int64_t(R) * NT;
        if (rb >= r0 + tile || rb >= n_pad) break;
        i = rb + R * int64_t(threadIdx.x);
        lv = row_len_pair<L8>(row_len, i < n_pad ? i : n_pad - R);
        base = addr.base(i < n_pad ? i : n_pad - R);
        if (i >= n_pad) lv = I{};
    }
    if (epi.dot) {
        // fixed-order workgroup sum: butterfly inside each wave, then the waves in order
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off);
        if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = dsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < NT / kWave; ++w) t += wsum[w];
            epi.dot[r0 / tile] = t;
        }
    }
}

// ---- pJDS with T lanes per row --------------------------------------------------------
// One wave per block of b_r = 64 / T sorted rows.  Lane l serves row l / T of the block and
// takes its entries t, t + T, t + 2T, ... (t = l % T); step q of the block is the 64-slot
// segment at block_start + 64 q, so each load of the wave is one contiguous segment for
// every T.  Row 0 of a block is its longest row, so lane 0 has an entry at every step of the
// block and serves as the lead lane.  The T partial sums of a row are combined by an xor
// butterfly: every lane of the row ends with the same sum, added in a fixed order, and the
// row's first lane writes y.
struct LanesAddr {                      // lane slot b (= block_start + lane), step q: b + 64 q
    int64_t start;
    __device__ int64_t base(int64_t lane) const { return start + lane; }
    __device__ int64_t operator()(int q, int64_t b) const { return b + int64_t(q) * kWave; }
};

template <class T, int TL>
__global__ __launch_bounds__(kBlock) void pjds_lanes_kernel(
    int64_t n_rows, int64_t n_blocks, const int32_t *__restrict__ row_len,
    const int64_t *__restrict__ offsets, const int32_t *__restrict__ col_p,
    const T *__restrict__ val_p, const int32_t *__restrict__ perm, const T *__restrict__ x, T *y,
    Epilogue<T> epi, uint32_t flags) {
    constexpr int BR = kWave / TL;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = int64_t(logical_block(flags)) * kWavesPerBlock + (threadIdx.x >> 6);
    if (b >= n_blocks) return;
    const int t = lane % TL;
    const int64_t i = b * BR + lane / TL;                    // < n_pad = n_blocks * BR
    const int len = row_len[i];
    const int steps = len > t ? (len - t + TL - 1) / TL : 0;
    const int64_t start = offsets[b];
    const int W = __builtin_amdgcn_readfirstlane(int((offsets[b + 1] - start) / kWave));
    T acc = row_range_sum(start + lane, start, steps, 0, W, LanesAddr{start}, col_p, val_p, XGlobal<T>{x, 1, 0});
#pragma unroll
    for (int off = 1; off < TL; off <<= 1) acc += __shfl_xor(acc, off);
    if (t == 0 && i < n_rows) {
        const int64_t r = (flags & PJDS_Y_PERMUTED) ? i : perm[i];
        epi.store(y, r, acc);
    }
}

__global__ void pack_lengths_kernel(const int32_t *__restrict__ rl, uint8_t *__restrict__ rl8, int64_t n) {
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x)
        rl8[k] = uint8_t(rl[k]);
}

__global__ void zero_ints_kernel(int32_t *p, int64_t n) {
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) p[k] = 0;
}

// ---- pJDS with k right-hand sides -----------------------------------------------------
// A tile covers LPR * VPL consecutive right-hand sides.  LPR consecutive lanes share one
// sorted row; each of them applies the row's entries to VPL adjacent right-hand sides, read
// from the interleaved X (X[c*k + v]) with one VPL-wide load.  A matrix entry is therefore
// loaded once per tile, a wave covers R = 64/LPR rows, and a gather instruction reads LPR *
// VPL contiguous values per row.  Tiles over k run in gridDim.y; with NVT = 2 each lane also
// takes the same place in the next vector tile (an even number of tiles and VPL = 4), so the
// matrix is streamed once per two tiles: for each entry it gathers two VPL-wide pieces of the
// X row and keeps two accumulators, with the same FMAs in the same order per (row, vector).
// Steps run in groups of U with two register sets in turn, so a group's value and index loads
// are in flight while the group before it gathers X.

template <class T, bool JD, int BR, int LPR, int VPL, int NVT>
__global__ __launch_bounds__(kBlock) void pjds_spmmv_kernel(
    int64_t n_rows, int64_t n_pad, int64_t n_waves, int32_t k,
    const int32_t *__restrict__ row_len, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ col_p, const T *__restrict__ val_p,
    const int32_t *__restrict__ perm, const T *__restrict__ X, T *__restrict__ Y, uint32_t flags) {
    typedef typename VecOf<T, VPL>::type V;
    constexpr int R = kWave / LPR;
    constexpr int U = NVT > 1 ? 2 : (VPL >= 4 ? 4 : kUnroll);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = int64_t(logical_block(flags)) * kWavesPerBlock + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    int v[NVT], vc[NVT];
#pragma unroll
    for (int n = 0; n < NVT; ++n) {
        v[n] = (int(blockIdx.y) * NVT + n) * (LPR * VPL) + (lane % LPR) * VPL;
        vc[n] = v[n] < k ? v[n] : k - VPL;
    }
    const int64_t i = w * R + lane / LPR;
    int len = row_len[i < n_pad ? i : n_pad - 1];        // clamped, then masked
    if (i >= n_pad) len = 0;
    const int m = wave_first(len);
    V acc[NVT];
#pragma unroll
    for (int n = 0; n < NVT; ++n)
#pragma unroll
        for (int q = 0; q < VPL; ++q) reinterpret_cast<T *>(&acc[n])[q] = T(0);
    if (m > 0) {
        const int64_t i_lead = w * R;
        const PjdsAddr<JD, BR> addr{offsets};
        const int64_t base = addr.base(i), base_lead = addr.base(i_lead);
        // two register sets of U steps in turn: a group's X gathers go out, then the next
        // group's value and index loads, then the group's FMAs
        T a_v[2][U];
        int32_t a_c[2][U];
        auto load = [&](int jb, int set) {
            int64_t a[U];                              // indices first, then values
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + u < m ? jb + u : m - 1;
                a[u] = addr(j, j < len ? base : base_lead);
                a_c[set][u] = ld_stream(col_p + a[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) a_v[set][u] = ld_stream(val_p + a[u]);
        };
        auto group = [&](int jb, int set) {
            V xv[U][NVT];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int n = 0; n < NVT; ++n)
                    xv[u][n] = *reinterpret_cast<const V *>(X + int64_t(a_c[set][u]) * k + vc[n]);
            if (jb + U < m) load(jb + U, set ^ 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool on = jb + u < len && jb + u < m;
#pragma unroll
                for (int n = 0; n < NVT; ++n)
#pragma unroll
                    for (int q = 0; q < VPL; ++q) {
                        T &aq = reinterpret_cast<T *>(&acc[n])[q];
                        const T s = __builtin_fma(a_v[set][u], reinterpret_cast<const T *>(&xv[u][n])[q], aq);
                        aq = on ? s : aq;
                    }
            }
        };
        load(0, 0);
        for (int jb = 0; jb < m; jb += 2 * U) {
            group(jb, 0);
            if (jb + U < m) group(jb + U, 1);
        }
    }
    if (i < n_rows) {
        const int64_t r = (flags & PJDS_Y_PERMUTED) ? i : perm[i];
#pragma unroll
        for (int n = 0; n < NVT; ++n)
            if (v[n] < k) __builtin_nontemporal_store(acc[n], reinterpret_cast<V *>(Y + r * k + v[n]));
    }
}

// ---- ELLPACK-R, Listing 1 -------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void ellr_spmv_kernel(
    int64_t n_rows, int64_t n_pad, const int32_t *__restrict__ rowmax,
    const int32_t *__restrict__ col_e, const T *__restrict__ val_e,
    const T *__restrict__ x, T *__restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int len = i < n_pad ? rowmax[i] : 0;
    const int m = wave_max(len);
    // lanes past their row read the slot of the wave's longest row (never padding)
    const int64_t i_lead = m > 0 ? i - (threadIdx.x & (kWave - 1)) + lead_lane(len, m) : 0;
    const T acc = row_range_sum(EllrAddr{n_pad}.base(i), i_lead, len, 0, m, EllrAddr{n_pad}, col_e, val_e,
                                XGlobal<T>{x, 1, 0});
    if (i < n_rows) y[i] = acc;
}

// ---- CSR --------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void csr_scalar_kernel(
    int64_t n_rows, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_rows) return;
    T acc = T(0);
    for (int64_t k = row_ptr[i], e = row_ptr[i + 1]; k < e; ++k)
        acc = __builtin_fma(val[k], x[col[k]], acc);
    y[i] = acc;
}

template <class T, int G>
__global__ __launch_bounds__(kBlock) void csr_vector_kernel(
    int64_t n_rows, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y) {
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t i = t / G;
    const int sub = int(t % G);
    T acc = T(0);
    if (i < n_rows)
        for (int64_t k = row_ptr[i] + sub, e = row_ptr[i + 1]; k < e; k += G)
            acc = __builtin_fma(val[k], x[col[k]], acc);
    // butterfly: every lane of the group ends with the same, order-fixed sum
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    if (i < n_rows && sub == 0) y[i] = acc;
}

// ---- bandwidth probes ---------------------------------------------------------------------
// Each workgroup streams its own contiguous chunk of the array with 16-byte loads,
// kProbeInFlight independent ones per thread and round, over kProbeBlocks workgroups (four per
// CU).  On an MI355X this layout read 2 GiB at 7.0 TB/s where a grid-strided one with four
// loads in flight reached 6.0: the chunks keep every workgroup on its own DRAM pages.
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int kProbeInFlight = 8;
constexpr int kProbeBlocks = 1024;

// [b0, b1): workgroup blockIdx.x's chunk of n2 16-byte elements
__device__ __forceinline__ void probe_chunk(int64_t n2, int64_t &b0, int64_t &b1) {
    const int64_t per = (n2 + gridDim.x - 1) / gridDim.x;
    b0 = min(int64_t(blockIdx.x) * per, n2);
    b1 = min(b0 + per, n2);
}

// Sum of n doubles, one partial sum per workgroup in out[blockIdx.x].  NT: non-temporal loads
// (the read ceiling); else ordinary loads that allocate in every cache level on the way (a pass
// that evicts what the caches held and leaves no dirty line behind).
template <bool NT>
__global__ __launch_bounds__(kBlock) void probe_read_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t n) {
    int64_t b0, b1;
    probe_chunk(n / 2, b0, b1);
    const dbl2 *in2 = reinterpret_cast<const dbl2 *>(in);
    dbl2 acc = {0.0, 0.0};
    for (int64_t k = b0 + threadIdx.x; k < b1; k += int64_t(kBlock) * kProbeInFlight) {
        dbl2 v[kProbeInFlight];
#pragma unroll
        for (int u = 0; u < kProbeInFlight; ++u) {
            const int64_t e = k + u * kBlock;
            v[u] = e < b1 ? (NT ? __builtin_nontemporal_load(in2 + e) : in2[e]) : dbl2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kProbeInFlight; ++u) acc += v[u];
    }
    double s = acc.x + acc.y;
    if (n & 1 && blockIdx.x == 0 && threadIdx.x == 0) s += in[n - 1];
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void probe_copy_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t n) {
    int64_t b0, b1;
    probe_chunk(n / 2, b0, b1);
    const dbl2 *in2 = reinterpret_cast<const dbl2 *>(in);
    dbl2 *out2 = reinterpret_cast<dbl2 *>(out);
    for (int64_t k = b0 + threadIdx.x; k < b1; k += int64_t(kBlock) * kProbeInFlight) {
        dbl2 v[kProbeInFlight];
#pragma unroll
        for (int u = 0; u < kProbeInFlight; ++u) {
            const int64_t e = k + u * kBlock;
            v[u] = e < b1 ? __builtin_nontemporal_load(in2 + e) : dbl2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kProbeInFlight; ++u) {
            const int64_t e = k + u * kBlock;
            if (e < b1) __builtin_nontemporal_store(v[u], out2 + e);
        }
    }
    if (n & 1 && blockIdx.x == 0 && threadIdx.x == 0) out[n - 1] = in[n - 1];
}

template <class T>
Epilogue<T> make_epi(const EpiArgs &a) {
    return Epilogue<T>{T(a.alpha), T(a.beta), static_cast<const T *>(a.z), static_cast<const T *>(a.beta_dev),
                       T(a.bscale), static_cast<const T *>(a.alpha_dev), a.dot_partial, a.norm_part,
                       a.n_norm, a.inv_prev, a.inv_out, a.beta_out};
}

int launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PJDS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return PJDS_OK;
}

int64_t ws_partials_bytes(const pjds_info &in, int32_t dtype) {
    const int64_t sz = dtype == PJDS_F64 ? 8 : 4;
    return (in.n_chunks * kWave * sz + 255) / 256 * 256;
}

template <class T, bool JD, int BR>
void launch_pjds(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp,
                 const void *vp, const int32_t *perm, const int32_t *sched, void *work,
                 const void *x, void *y, const EpiArgs &ea, uint32_t flags, hipStream_t s) {
    const int64_t groups = ceil_div(in.n_pad, kWave);
    const int64_t waves = in.n_chunks + groups;
    const dim3 grid(unsigned(ceil_div(waves, kWavesPerBlock)));
    T *partials = static_cast<T *>(work);
    int32_t *counters = work ? reinterpret_cast<int32_t *>(static_cast<char *>(work) + ws_partials_bytes(in, sizeof(T) == 8 ? PJDS_F64 : PJDS_F32)) : nullptr;
    launch_main((pjds_spmv_kernel<T, JD, BR>), grid, dim3(kBlock), 0, s, in.n_rows, in.n_pad,
                       groups, in.n_chunks, in.split_len, rl, off, cp, static_cast<const T *>(vp),
                       perm, sched, partials, counters, static_cast<const T *>(x),
                       static_cast<T *>(y), make_epi<T>(ea), flags);
}

template <class T, bool JD, int BR>
void launch_pjds2(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp, const void *vp,
                  const int32_t *perm, const void *x, void *y, const EpiArgs &ea, uint32_t flags, hipStream_t s) {
    const int64_t waves = ceil_div(in.n_pad, int64_t(kWave) * kRowsPerLane);
    const dim3 grid(unsigned(ceil_div(waves, kWavesPerBlock)));
    launch_main((pjds_spmv2_kernel<T, JD, BR>), grid, dim3(kBlock), 0, s, in.n_rows, in.n_pad, waves, rl, off,
                       cp, static_cast<const T *>(vp), perm, static_cast<const T *>(x), static_cast<T *>(y),
                       make_epi<T>(ea), flags);
}

template <class T, bool JD, int BR, int LPR, int VPL>
void launch_spmmv_lv(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp,
                     const void *vp, const int32_t *perm, int32_t k, const void *X, void *Y,
                     uint32_t flags, hipStream_t s) {
    const int64_t waves = ceil_div(in.n_pad, kWave / LPR);
    const int64_t tiles = ceil_div(k, LPR * VPL);
    if (tiles % 2 == 0 && VPL >= 4) {
        // two vector tiles per lane: the matrix is streamed once per pair of tiles
        const dim3 grid(unsigned(ceil_div(waves, kWavesPerBlock)), unsigned(tiles / 2));
        launch_main((pjds_spmmv_kernel<T, JD, BR, LPR, VPL, 2>), grid, dim3(kBlock), 0, s, in.n_rows,
                           in.n_pad, waves, k, rl, off, cp, static_cast<const T *>(vp), perm,
                           static_cast<const T *>(X), static_cast<T *>(Y), flags);
        return;
    }
    const dim3 grid(unsigned(ceil_div(waves, kWavesPerBlock)), unsigned(tiles));
    launch_main((pjds_spmmv_kernel<T, JD, BR, LPR, VPL, 1>), grid, dim3(kBlock), 0, s, in.n_rows,
                       in.n_pad, waves, k, rl, off, cp, static_cast<const T *>(vp), perm,
                       static_cast<const T *>(X), static_cast<T *>(Y), flags);
}

template <class T, bool JD, int BR, int VPL>
void launch_spmmv_v(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp,
                    const void *vp, const int32_t *perm, int32_t k, int32_t lpr, const void *X,
                    void *Y, uint32_t flags, hipStream_t s) {
    switch (lpr) {
        case 1: launch_spmmv_lv<T, JD, BR, 1, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
        case 2: launch_spmmv_lv<T, JD, BR, 2, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
        case 4: launch_spmmv_lv<T, JD, BR, 4, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
        case 8: launch_spmmv_lv<T, JD, BR, 8, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
        case 16: launch_spmmv_lv<T, JD, BR, 16, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
        default: launch_spmmv_lv<T, JD, BR, 32, VPL>(in, rl, off, cp, vp, perm, k, X, Y, flags, s); break;
    }
}

template <class T, bool JD, int BR>
void launch_spmmv(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp,
                  const void *vp, const int32_t *perm, int32_t k, int32_t t, int32_t vpl, const void *X,
                  void *Y, uint32_t flags, hipStream_t s) {
    const int32_t lpr = t / vpl;
    if (vpl == 1) launch_spmmv_v<T, JD, BR, 1>(in, rl, off, cp, vp, perm, k, lpr, X, Y, flags, s);
    else if (vpl == 2) launch_spmmv_v<T, JD, BR, 2>(in, rl, off, cp, vp, perm, k, lpr, X, Y, flags, s);
    else launch_spmmv_v<T, JD, BR, 4>(in, rl, off, cp, vp, perm, k, lpr, X, Y, flags, s);
}

int32_t lanes_of(const pjds_info &in) { return int32_t(1) << ((in.flags & PJDS_LANES_MASK) >> PJDS_LANES_SHIFT); }

template <class T>
void launch_lanes(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp, const void *vp,
                  const int32_t *perm, const void *x, void *y, const EpiArgs &ea, uint32_t flags, hipStream_t s) {
    const dim3 grid(unsigned(ceil_div(in.n_blocks, kWavesPerBlock)));
#define PJDS_LANES_CASE(TL)                                                                              \
    launch_main((pjds_lanes_kernel<T, TL>), grid, dim3(kBlock), 0, s, in.n_rows, in.n_blocks, rl, off,        \
                       cp, static_cast<const T *>(vp), perm, static_cast<const T *>(x), static_cast<T *>(y),    \
                       make_epi<T>(ea), flags)
    switch (lanes_of(in)) {
        case 2: PJDS_LANES_CASE(2); break;
        case 4: PJDS_LANES_CASE(4); break;
        case 8: PJDS_LANES_CASE(8); break;
        case 16: PJDS_LANES_CASE(16); break;
        case 32: PJDS_LANES_CASE(32); break;
        default: PJDS_LANES_CASE(64); break;
    }
#undef PJDS_LANES_CASE
}

// Dispatch on (dtype, layout, block height) to a compile-time instantiation.
template <template <class, bool, int> class K, class... A>
void dispatch(int32_t dtype, bool jd, int32_t br, A &&...a) {
    auto go = [&](auto tag) {
        using T = decltype(tag);
        if (jd) {
            if (br == 32) K<T, true, 32>::run(a...);
            else if (br == 64) K<T, true, 64>::run(a...);
            else K<T, true, 128>::run(a...);
        } else {
            if (br == 32) K<T, false, 32>::run(a...);
            else if (br == 64) K<T, false, 64>::run(a...);
            else K<T, false, 128>::run(a...);
        }
    };
    if (dtype == PJDS_F64) go(double{});
    else go(float{});
}

template <class T, bool JD, int BR>
struct SpmvK {
    template <class... A>
    static void run(A &&...a) { launch_pjds<T, JD, BR>(a...); }
};
template <class T, bool JD, int BR>
struct Spmv2K {
    template <class... A>
    static void run(A &&...a) { launch_pjds2<T, JD, BR>(a...); }
};
// The single-vector product for any pJDS matrix: T lanes per row, or one lane per row.
void launch_product(const pjds_info &in, const int32_t *rl, const int64_t *off, const int32_t *cp, const void *vp,
                    const int32_t *perm, const int32_t *sched, void *work, int32_t dtype, const void *x, void *y,
                    const EpiArgs &ea, uint32_t flags, hipStream_t s) {
    if (lanes_of(in) > 1) {
        if (dtype == PJDS_F64) launch_lanes<double>(in, rl, off, cp, vp, perm, x, y, ea, flags, s);
        else launch_lanes<float>(in, rl, off, cp, vp, perm, x, y, ea, flags, s);
        return;
    }
    if (flags & PJDS_TWO_ROWS) {
        dispatch<Spmv2K>(dtype, !(in.flags & PJDS_LAYOUT_BLOCK), in.block_height, in, rl, off, cp, vp, perm, x, y, ea,
                         flags, s);
        return;
    }
    dispatch<SpmvK>(dtype, !(in.flags & PJDS_LAYOUT_BLOCK), in.block_height, in, rl, off, cp, vp, perm, sched, work,
                    x, y, ea, flags, s);
}

// Whether the plain product can take two rows per lane: no long-row work items, one lane per
// row, and a sort that keeps whole 64 R-row groups sorted.
int check_two_rows(const pjds_info &in) {
    if (in.n_chunks) return fail(PJDS_ERR_UNSUPPORTED, "two rows per lane with long-row work items (convert with split_len < 0)");
    if (lanes_of(in) > 1) return fail(PJDS_ERR_UNSUPPORTED, "two rows per lane with several lanes per row");
    const int64_t group = int64_t(kWave) * kRowsPerLane;
    if (in.sort_window < in.n_rows && in.sort_window % group)
        return fail(PJDS_ERR_ARG, "two rows per lane need a sort window that is a multiple of %lld", (long long)group);
    return PJDS_OK;
}

template <class T, bool JD, int BR>
struct SpmmvK {
    template <class... A>
    static void run(A &&...a) { launch_spmmv<T, JD, BR>(a...); }
};

int check_info(const pjds_info *info, int32_t dtype) {
    if (!info) return fail(PJDS_ERR_ARG, "info is NULL");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    const int32_t br = info->block_height, lanes = lanes_of(*info);
    if (lanes > 1 ? (br * lanes != kWave || !(info->flags & PJDS_LAYOUT_BLOCK) || info->n_chunks)
                  : (br != 32 && br != 64 && br != 128))
        return fail(PJDS_ERR_ARG, "block_height %d with %d lanes per row", br, lanes);
    if (info->n_rows < 0 || info->n_pad < info->n_rows || info->n_pad % br) return fail(PJDS_ERR_ARG, "inconsistent info");
    return PJDS_OK;
}

}  // namespace

int check_product_info(const pjds_info *info, int32_t dtype) { return check_info(info, dtype); }

int check_xlds(const pjds_info &in, int32_t dtype, int32_t x_halo, int32_t tile_rows) {
    if (lanes_of(in) > 1) return fail(PJDS_ERR_UNSUPPORTED, "x staging with several lanes per row");
    const int64_t w = in.sort_window;
    if (!(in.flags & PJDS_LAYOUT_BLOCK) || w >= in.n_rows || w % kBlock)
        return fail(PJDS_ERR_ARG, "x staging needs the block layout and a sort window that is a multiple of %d", kBlock);
    if (x_halo < 0) return fail(PJDS_ERR_ARG, "x_halo %d", x_halo);
    const int64_t tile = tile_rows == 0 ? std::max<int64_t>(w, 1024) : tile_rows;
    if (tile < kBlock || tile % kBlock || (tile % w && w % tile))
        return fail(PJDS_ERR_ARG, "tile_rows %lld: a multiple of %d that divides or is divided by the sort window", (long long)tile, kBlock);
    const int64_t tsize = dtype == PJDS_F64 ? 8 : 4;
    const int64_t cap = std::min<int64_t>(std::max(tile, w) + 2 * int64_t(x_halo), in.n_cols);
    if (cap * tsize > 64 * 1024) return fail(PJDS_ERR_ARG, "x range of %lld entries exceeds 64 KiB of LDS", (long long)cap);
    return PJDS_OK;
}

int64_t xlds_tiles(const pjds_info &in, int32_t tile_rows) {
    const int64_t tile = tile_rows == 0 ? std::max<int64_t>(in.sort_window, 1024) : tile_rows;
    return ceil_div(in.n_pad, tile);
}

void launch_xlds(const pjds_info &in, const int32_t *d_row_len, const int64_t *d_offsets, const int32_t *d_col_p,
                 const void *d_val_p, const int32_t *d_perm, int32_t dtype, const void *d_x, void *d_y,
                 int32_t x_halo, int32_t tile_rows, const EpiArgs &ea, uint32_t flags, hipStream_t s) {
    const int64_t w = in.sort_window;
    const int64_t tile = tile_rows == 0 ? std::max<int64_t>(w, 1024) : tile_rows;
    const int64_t tsize = dtype == PJDS_F64 ? 8 : 4;
    const int64_t cap = std::min<int64_t>(std::max(tile, w) + 2 * int64_t(x_halo), in.n_cols);
    const dim3 grid(unsigned(ceil_div(in.n_pad, tile)));
    const size_t lds = size_t(std::max<int64_t>(cap, 1) * tsize);
    // 512 threads when the tile is a multiple of 512 rows, else 256 (1024-thread workgroups
    // measured slower: longer waits at the barrier, fewer workgroups per CU); with two rows
    // per lane, half as many threads as rows per tile, at most 512
    const bool two = flags & PJDS_TWO_ROWS;
    const int64_t per = two ? tile / kRowsPerLane : tile;     // threads the tile could use
    const int nt = two ? (per % 512 == 0 ? 512 : per % 256 == 0 ? 256 : 128) : tile % 512 == 0 ? 512 : kBlock;
    auto go = [&](auto tag, auto l8) {
        using T = decltype(tag);
        constexpr bool L8 = decltype(l8)::value;
        const int br = in.block_height;
        if (two) {
#define PJDS_XLDS2_LAUNCH(B, N)                                                                           \
            launch_main((pjds_spmv_lds2_kernel<T, B, N, L8>), grid, dim3(N), lds, s, in.n_rows, in.n_cols,        \
                               in.n_pad, w, int64_t(x_halo), tile, d_row_len, d_offsets, d_col_p,              \
                               static_cast<const T *>(d_val_p), d_perm, static_cast<const T *>(d_x),          \
                               static_cast<T *>(d_y), make_epi<T>(ea), flags)
#define PJDS_XLDS2_CASE(B)                                                                                \
            if (nt == 512) PJDS_XLDS2_LAUNCH(B, 512);                                                      \
            else if (nt == 256) PJDS_XLDS2_LAUNCH(B, 256);                                                 \
            else PJDS_XLDS2_LAUNCH(B, 128)
            if (br == 32) { PJDS_XLDS2_CASE(32); }
            else if (br == 64) { PJDS_XLDS2_CASE(64); }
            else { PJDS_XLDS2_CASE(128); }
#undef PJDS_XLDS2_CASE
#undef PJDS_XLDS2_LAUNCH
            return;
        }
#define PJDS_XLDS_LAUNCH(B, N)                                                                            \
        launch_main((pjds_spmv_lds_kernel<T, B, N, L8>), grid, dim3(N), lds, s, in.n_rows, in.n_cols,        \
                           in.n_pad, w, int64_t(x_halo), tile, d_row_len, d_offsets, d_col_p,                  \
                           static_cast<const T *>(d_val_p), d_perm, static_cast<const T *>(d_x),              \
                           static_cast<T *>(d_y), make_epi<T>(ea), flags)
#define PJDS_XLDS_CASE(B)                                                                                 \
        if (nt == 512) PJDS_XLDS_LAUNCH(B, 512);                                                           \
        else PJDS_XLDS_LAUNCH(B, kBlock)
        if (br == 32) { PJDS_XLDS_CASE(32); }
        else if (br == 64) { PJDS_XLDS_CASE(64); }
        else { PJDS_XLDS_CASE(128); }
#undef PJDS_XLDS_CASE
#undef PJDS_XLDS_LAUNCH
    };
    const bool len8 = flags & PJDS_ROW_LEN8;
    if (dtype == PJDS_F64) {
        if (len8) go(double{}, std::true_type{});
        else go(double{}, std::false_type{});
    } else {
        if (len8) go(float{}, std::true_type{});
        else go(float{}, std::false_type{});
    }
}

void launch_spmv_epi(const pjds_info &in, const int32_t *d_row_len, const int64_t *d_offsets,
                     const int32_t *d_col_p, const void *d_val_p, const int32_t *d_sched, void *d_work,
                     int32_t dtype, const void *d_x, void *d_y, const EpiArgs &ea, uint32_t flags,
                     hipStream_t s) {
    launch_product(in, d_row_len, d_offsets, d_col_p, d_val_p, nullptr, d_sched, d_work, dtype, d_x, d_y, ea, flags, s);
}

// ---- fixed device scratch of pjds_spmv_noalloc -----------------------------------------
// The long-row partial sums and completion counters of that entry point live here, in the
// code object's own device memory, so the call allocates nothing.  In host code `scratch` only
// names the variable: its device address, different on each GPU, comes from
// hipGetSymbolAddress with that GPU current, and only that address goes to kernels.
static __device__ __align__(256) unsigned char scratch[PJDS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PJDS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(PJDS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PJDS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PJDS_OK;
}

namespace {
thread_local LaunchEvents g_launch_events{nullptr, nullptr};
}  // namespace

LaunchEvents take_launch_events() {
    const LaunchEvents e = g_launch_events;
    g_launch_events = LaunchEvents{nullptr, nullptr};
    return e;
}

}  // namespace pjds

using namespace pjds;

extern "C" {

int pjds_workspace_size(const pjds_info *info, int32_t dtype, int64_t *bytes) {
    if (int rc = check_info(info, dtype)) return rc;
    if (!bytes) return fail(PJDS_ERR_ARG, "bytes is NULL");
    *bytes = info->n_chunks ? ws_partials_bytes(*info, dtype) + (info->n_chunks * 4 + 255) / 256 * 256 : 0;
    return PJDS_OK;
}

int pjds_workspace_init(const pjds_info *info, int32_t dtype, void *d_work, void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (!info->n_chunks) return PJDS_OK;
    if (!d_work) return fail(PJDS_ERR_ARG, "d_work is NULL");
    int32_t *counters = reinterpret_cast<int32_t *>(static_cast<char *>(d_work) + ws_partials_bytes(*info, dtype));
    const int64_t n = info->n_chunks;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(unsigned(std::min<int64_t>(ceil_div(n, kBlock), 1024))), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), counters, n);
    return launch_status("pjds_workspace_init");
}

int pjds_spmv(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
              const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
              const int32_t *d_sched, void *d_work, int32_t dtype, const void *d_x, void *d_y,
              uint32_t flags, void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (flags & ~(PJDS_Y_PERMUTED | PJDS_XCD_REMAP | PJDS_TWO_ROWS))
        return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (flags & PJDS_TWO_ROWS)
        if (int rc = check_two_rows(*info)) return rc;
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p || !d_x)) return fail(PJDS_ERR_ARG, "NULL device array");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter y)");
    if (info->n_chunks && (!d_sched || !d_work)) return fail(PJDS_ERR_ARG, "long rows need d_sched and d_work");
    launch_product(*info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched, d_work, dtype, d_x, d_y,
                   EpiArgs{}, flags, static_cast<hipStream_t>(stream));
    return launch_status("pjds_spmv");
}

int pjds_spmv_noalloc(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                      const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                      const int32_t *d_sched, int32_t dtype, const void *d_x, void *d_y,
                      uint32_t flags, void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (flags & ~(PJDS_Y_PERMUTED | PJDS_XCD_REMAP | PJDS_TWO_ROWS))
        return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (flags & PJDS_TWO_ROWS)
        if (int rc = check_two_rows(*info)) return rc;
    const int64_t partial_bytes = ws_partials_bytes(*info, dtype);
    const int64_t need = info->n_chunks ? partial_bytes + (info->n_chunks * 4 + 255) / 256 * 256 : 0;
    if (need > PJDS_NOALLOC_SCRATCH_BYTES)
        return fail(PJDS_ERR_OVERFLOW, "long-row workspace of %lld bytes exceeds the fixed scratch of %lld bytes",
                    (long long)need, (long long)PJDS_NOALLOC_SCRATCH_BYTES);
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p || !d_x)) return fail(PJDS_ERR_ARG, "NULL device array");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter y)");
    if (info->n_chunks && !d_sched) return fail(PJDS_ERR_ARG, "long rows need d_sched");
    void *work = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (info->n_chunks) {
        if (int rc = scratch_address(&work)) return rc;
        // the counters must start at zero whatever an earlier call left behind
        int32_t *counters = reinterpret_cast<int32_t *>(static_cast<char *>(work) + partial_bytes);
        const int64_t n = info->n_chunks;
        hipLaunchKernelGGL(zero_ints_kernel, dim3(unsigned(std::min<int64_t>(ceil_div(n, kBlock), 1024))), dim3(kBlock), 0,
                           s, counters, n);
        if (int rc = launch_status("pjds_spmv_noalloc (clearing counters)")) return rc;
    }
    launch_product(*info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched, work, dtype, d_x, d_y,
                   EpiArgs{}, flags, s);
    return launch_status("pjds_spmv_noalloc");
}

int pjds_spmv_axpby(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                    const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                    const int32_t *d_sched, void *d_work, int32_t dtype, const void *d_x,
                    double alpha, double beta, const void *d_z, void *d_y, uint32_t flags,
                    void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (flags & ~(PJDS_Y_PERMUTED | PJDS_XCD_REMAP)) return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p || !d_x)) return fail(PJDS_ERR_ARG, "NULL device array");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter y)");
    if (info->n_chunks && (!d_sched || !d_work)) return fail(PJDS_ERR_ARG, "long rows need d_sched and d_work");
    if (d_z && d_z != d_y && d_z == d_x) return fail(PJDS_ERR_ARG, "z may be y but not x");
    EpiArgs ea{alpha, beta, d_z, nullptr, 0.0};
    launch_product(*info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched, d_work, dtype, d_x, d_y,
                   ea, flags, static_cast<hipStream_t>(stream));
    return launch_status("pjds_spmv_axpby");
}

int pjds_spmmv(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
               const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
               int32_t dtype, int32_t k, int32_t vectors_per_tile, int32_t vectors_per_lane,
               const void *d_X, void *d_Y, uint32_t flags, void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (flags & ~(PJDS_Y_PERMUTED | PJDS_XCD_REMAP)) return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (lanes_of(*info) > 1) return fail(PJDS_ERR_UNSUPPORTED, "SpMMV with several lanes per row");
    if (k < 1) return fail(PJDS_ERR_ARG, "k = %d", k);
    const int32_t t = vectors_per_tile, vpl = vectors_per_lane;
    if (vpl != 1 && vpl != 2 && vpl != 4) return fail(PJDS_ERR_ARG, "vectors_per_lane %d: must be 1, 2 or 4", vpl);
    if (k % vpl) return fail(PJDS_ERR_ARG, "k = %d must be a multiple of vectors_per_lane %d", k, vpl);
    const int32_t lpr = vpl ? t / vpl : 0;
    if (t % vpl || (lpr != 1 && lpr != 2 && lpr != 4 && lpr != 8 && lpr != 16 && lpr != 32))
        return fail(PJDS_ERR_ARG, "vectors_per_tile %d: vectors_per_lane times 1, 2, 4, 8, 16 or 32", t);
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_Y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p || !d_X)) return fail(PJDS_ERR_ARG, "NULL device array");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter Y)");
    const int64_t elt = dtype == PJDS_F64 ? 8 : 4;
    if ((reinterpret_cast<uintptr_t>(d_X) | reinterpret_cast<uintptr_t>(d_Y)) % uintptr_t(elt * vpl))
        return fail(PJDS_ERR_ARG, "X and Y must be aligned to vectors_per_lane values");
    if (ceil_div(k, t) > 65535) return fail(PJDS_ERR_ARG, "too many vector tiles");
    dispatch<SpmmvK>(dtype, !(info->flags & PJDS_LAYOUT_BLOCK), info->block_height, *info, d_row_len,
                     d_offsets, d_col_p, d_val_p, d_perm, k, t, vpl, d_X, d_Y, flags,
                     static_cast<hipStream_t>(stream));
    return launch_status("pjds_spmmv");
}

int pjds_spmv_xlds(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                   const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm, int32_t dtype,
                   const void *d_x, void *d_y, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                   void *stream) {
    if (int rc = check_info(info, dtype)) return rc;
    if (flags & ~(PJDS_Y_PERMUTED | PJDS_XCD_REMAP | PJDS_TWO_ROWS | PJDS_ROW_LEN8))
        return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (int rc = pjds::check_xlds(*info, dtype, x_halo, tile_rows)) return rc;
    if ((flags & PJDS_ROW_LEN8) && info->max_row_len > 255)
        return fail(PJDS_ERR_UNSUPPORTED, "PJDS_ROW_LEN8 with rows of %d entries (at most 255)", info->max_row_len);
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p)) return fail(PJDS_ERR_ARG, "NULL device array");
    // every tile copies its range of x into LDS, even when the matrix has no entries
    if (info->n_cols && !d_x) return fail(PJDS_ERR_ARG, "d_x is NULL");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter y)");
    pjds::launch_xlds(*info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, dtype, d_x, d_y, x_halo, tile_rows,
                      EpiArgs{}, flags, static_cast<hipStream_t>(stream));
    return launch_status("pjds_spmv_xlds");
}

int pjds_pack_lengths(const pjds_info *info, const int32_t *d_row_len, uint8_t *d_row_len8, void *stream) {
    if (!info) return fail(PJDS_ERR_ARG, "info is NULL");
    if (info->n_pad < info->n_rows || info->n_rows < 0) return fail(PJDS_ERR_ARG, "inconsistent info");
    if (info->max_row_len > 255)
        return fail(PJDS_ERR_UNSUPPORTED, "rows of %d entries do not fit one byte", info->max_row_len);
    if (info->n_pad == 0) return PJDS_OK;
    if (!d_row_len || !d_row_len8) return fail(PJDS_ERR_ARG, "NULL device array");
    const int64_t n = info->n_pad;
    hipLaunchKernelGGL(pack_lengths_kernel, dim3(unsigned(std::min<int64_t>(ceil_div(n, kBlock), 4096))), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), d_row_len, d_row_len8, n);
    return launch_status("pjds_pack_lengths");
}

int ellr_spmv(const pjds_info *info, const int32_t *d_rowmax, const int32_t *d_col_e,
              const void *d_val_e, int32_t dtype, const void *d_x, void *d_y, void *stream) {
    if (!info) return fail(PJDS_ERR_ARG, "info is NULL");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    if (info->n_pad % kWave || info->n_pad < info->n_rows) return fail(PJDS_ERR_ARG, "inconsistent ELLPACK-R info");
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_rowmax || !d_y || (info->nnz_stored && (!d_col_e || !d_val_e || !d_x))) return fail(PJDS_ERR_ARG, "NULL device array");
    const dim3 grid(unsigned(ceil_div(info->n_pad, kBlock)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == PJDS_F64)
        launch_main(ellr_spmv_kernel<double>, grid, dim3(kBlock), 0, s, info->n_rows, info->n_pad, d_rowmax,
                           d_col_e, static_cast<const double *>(d_val_e), static_cast<const double *>(d_x), static_cast<double *>(d_y));
    else
        launch_main(ellr_spmv_kernel<float>, grid, dim3(kBlock), 0, s, info->n_rows, info->n_pad, d_rowmax,
                           d_col_e, static_cast<const float *>(d_val_e), static_cast<const float *>(d_x), static_cast<float *>(d_y));
    return launch_status("ellr_spmv");
}

int csr_spmv(int64_t n_rows, int64_t n_cols, const int64_t *d_row_ptr, const int32_t *d_col,
             const void *d_val, int32_t dtype, const void *d_x, void *d_y, int32_t variant, void *stream) {
    if (n_rows < 0 || n_cols < 0) return fail(PJDS_ERR_ARG, "negative size");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    if (variant != 1 && variant != 4 && variant != 16 && variant != 64) return fail(PJDS_ERR_ARG, "variant %d: must be 1, 4, 16 or 64", variant);
    if (n_rows == 0) return PJDS_OK;
    if (!d_row_ptr || !d_y) return fail(PJDS_ERR_ARG, "NULL device array");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t threads = n_rows * variant;
    if (ceil_div(threads, kBlock) > INT32_MAX) return fail(PJDS_ERR_OVERFLOW, "grid too large");
    const dim3 grid(unsigned(ceil_div(threads, kBlock)));
    auto go = [&](auto tag) {
        using T = decltype(tag);
        const T *v = static_cast<const T *>(d_val);
        const T *x = static_cast<const T *>(d_x);
        T *y = static_cast<T *>(d_y);
        switch (variant) {
            case 1: launch_main(csr_scalar_kernel<T>, grid, dim3(kBlock), 0, s, n_rows, d_row_ptr, d_col, v, x, y); break;
            case 4: launch_main((csr_vector_kernel<T, 4>), grid, dim3(kBlock), 0, s, n_rows, d_row_ptr, d_col, v, x, y); break;
            case 16: launch_main((csr_vector_kernel<T, 16>), grid, dim3(kBlock), 0, s, n_rows, d_row_ptr, d_col, v, x, y); break;
            default: launch_main((csr_vector_kernel<T, 64>), grid, dim3(kBlock), 0, s, n_rows, d_row_ptr, d_col, v, x, y); break;
        }
    };
    if (dtype == PJDS_F64) go(double{});
    else go(float{});
    return launch_status("csr_spmv");
}

int pjds_time_next_launch(void *start_event, void *stop_event) {
    if (!start_event != !stop_event) return fail(PJDS_ERR_ARG, "pjds_time_next_launch: both events or neither");
    g_launch_events = LaunchEvents{static_cast<hipEvent_t>(start_event), static_cast<hipEvent_t>(stop_event)};
    return PJDS_OK;
}

int pjds_probe(int32_t mode, const double *d_in, double *d_out, int64_t n, void *stream) {
    if ((mode != 0 && mode != 1 && mode != 2) || n < 0 || !d_in || !d_out) return fail(PJDS_ERR_ARG, "bad probe arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(static_cast<unsigned>(kProbeBlocks));
    if (mode == 0) launch_main(probe_read_kernel<true>, grid, dim3(kBlock), 0, s, d_in, d_out, n);
    else if (mode == 2) launch_main(probe_read_kernel<false>, grid, dim3(kBlock), 0, s, d_in, d_out, n);
    else launch_main(probe_copy_kernel, grid, dim3(kBlock), 0, s, d_in, d_out, n);
    return launch_status("pjds_probe");
}

}  // extern "C"
