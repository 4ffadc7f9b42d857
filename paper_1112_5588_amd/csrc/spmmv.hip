// SpMMV with the right-hand sides staged in LDS: Y = A X for k vectors, X and Y row-major
// (X[c * k + v]), the matrix in pJDS block layout sorted in windows (Sect. 2.1; applying each
// matrix entry to several right-hand sides is an extension beyond the paper's single vector).
//
// A workgroup owns `tile` consecutive sorted rows.  Sorting never moves a row out of its window
// of original rows, so the tile's rows lie in the original rows of the windows it touches; the
// workgroup copies those rows of X (widened by a halo on each side, clipped to the matrix and to
// the LDS cap), for the t vectors of its vector tile, into LDS once.  Then each wave runs
// 64 / LPR rows at a time exactly as pjds_spmmv does (LPR lanes per row, VPL contiguous vectors
// per lane, the same FMAs in the same order), reading an X row from LDS when it was staged and
// from global memory otherwise.  Results equal pjds_spmmv's bit for bit.
//
// Latency: the first group of matrix steps of a wave's first rows is loaded before X is
// written into LDS (its loads are in flight across the copy and the barrier), and the row loop
// keeps two register sets of matrix steps, loading the next group before the FMAs of the
// current one, so a group's matrix loads overlap the previous group's gathers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "launch.h"

namespace pjds {
namespace {

constexpr int kThreads = 512;            // threads of a workgroup
constexpr int kStage = 8;                // X values in flight per thread while staging
constexpr int64_t kMaxLds = 64 * 1024;   // staged X per workgroup (two workgroups per CU)


template <class T, int BR, int LPR, int VPL>
__global__ __launch_bounds__(kThreads) void spmmv_xlds_kernel(
    int64_t n_rows, int64_t n_cols, int64_t n_pad, int64_t window, int64_t halo, int64_t tile, int32_t cap,
    int32_t k, const int32_t *__restrict__ row_len, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ col_p, const T *__restrict__ val_p, const int32_t *__restrict__ perm,
    const T *__restrict__ X, T *__restrict__ Y, uint32_t flags) {
    typedef typename VecOf<T, VPL>::type V;
    constexpr int TV = LPR * VPL;                  // vectors of one vector tile
    constexpr int RW = kWave / LPR;                // rows of a wave
    constexpr int RP = kThreads / LPR;             // rows of the workgroup per pass
    constexpr int U = VPL >= 4 ? 4 : 8;            // entries in flight per lane
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    const int v0 = int(blockIdx.y) * TV;           // first vector of the tile
    const int64_t r0 = int64_t(xcd_group(blockIdx.x, gridDim.x)) * tile;
    const int64_t r1 = min(r0 + tile, n_pad);
    const int64_t lo_r = r0 / window * window;
    const int64_t hi_r = (r1 + window - 1) / window * window;
    const int64_t lo = max(lo_r - halo, int64_t(0));
    const int64_t hi = min(hi_r + halo, n_cols);
    const int32_t nr = int32_t(max(min(hi - lo, int64_t(cap)), int64_t(0)));   // staged X rows
    const int lane = threadIdx.x & (kWave - 1);
    // this lane's first vector; k is a multiple of VPL, so a lane's VPL values are all inside
    // [0, k) or all outside (then it computes a copy of the last VPL vectors and stores nothing)
    const int v = v0 + (lane % LPR) * VPL;
    const int vc = v < k ? v : k - VPL;
    const int q0 = vc - v0;                        // offset of the lane's values in a staged row
    // the rows of a pass: lengths and offsets, then (after the copy's loads are out) the first
    // group of matrix steps, in flight across the copy into LDS and the barrier
    T av[2][U];
    int32_t ac[2][U];
    int64_t rb = r0 + int64_t(threadIdx.x >> 6) * RW;
    int64_t i = rb + lane / LPR;
    const int64_t ia0 = i < n_pad ? i : n_pad - 1;
    int len = row_len[ia0];                              // clamped, then masked
    int64_t base = offsets[ia0 / BR] + (ia0 % BR);
    if (i >= n_pad) len = 0;
    auto load_grp = [&](int jb, int m_, int64_t bl, T (&a_v)[U], int32_t (&a_c)[U]) {
        int64_t a[U];                                    // indices first, then values
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = jb + u < m_ ? jb + u : m_ - 1;     // uniform clamp past the longest row
            a[u] = (j < len ? base : bl) + int64_t(j) * BR;
            a_c[u] = ld_stream(col_p + a[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) a_v[u] = ld_stream(val_p + a[u]);
    };
    // xs[r * TV + q] = X[(lo + r) * k + v0 + q]; vectors at or past k are staged as 0
    const int32_t total = nr * TV;
    // the first kPre chunks of the copy in registers, then the first matrix group, then the
    // LDS writes: all of these loads are in flight together
    constexpr int kPre = 2;
    {
        T sv[kPre * kStage];
#pragma unroll
        for (int u = 0; u < kPre * kStage; ++u) {
            const int32_t e = u * kThreads + int32_t(threadIdx.x);
            const int32_t r = e / TV, q = e % TV;
            sv[u] = e < total && v0 + q < k ? X[(lo + r) * k + v0 + q] : T(0);
        }
        const int m0 = wave_first(len);
        if (rb < r1 && m0 > 0) load_grp(0, m0, wave_first(base), av[0], ac[0]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kPre * kStage; ++u) {
            const int32_t e = u * kThreads + int32_t(threadIdx.x);
            if (e < total) xs[e] = sv[u];
        }
    }
    for (int32_t e0 = kThreads * kStage * kPre; e0 < total; e0 += kThreads * kStage) {
        T vv[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int32_t e = e0 + u * kThreads + int32_t(threadIdx.x);
            const int32_t r = e / TV, q = e % TV;
            vv[u] = e < total && v0 + q < k ? X[(lo + r) * k + v0 + q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int32_t e = e0 + u * kThreads + int32_t(threadIdx.x);
            if (e < total) xs[e] = vv[u];
        }
    }
    __syncthreads();
    for (bool first = true; rb < r1; rb += RP, first = false) {
        if (!first) {
            i = rb + lane / LPR;
            const int64_t ia = i < n_pad ? i : n_pad - 1;     // lanes past n_pad never use it
            len = row_len[ia];
            base = offsets[ia / BR] + (ia % BR);
            if (i >= n_pad) len = 0;
        }
        const int m = wave_first(len);
        const int64_t base_lead = wave_first(base);         // the wave's first row is its longest
        V acc;
#pragma unroll
        for (int q = 0; q < VPL; ++q) reinterpret_cast<T *>(&acc)[q] = T(0);
        if (m > 0) {
            if (!first) load_grp(0, m, base_lead, av[0], ac[0]);
            // two register sets in turn: the next group's matrix loads go out before this
            // group's FMAs, so they are in flight while the gathers are waited for
            auto grp = [&](int jb, int cur) {
                V xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    xv[u] = staged_or_global<V>(xs + q0, uint32_t(ac[cur][u]) - uint32_t(lo), uint32_t(nr), LPR, X,
                                                int64_t(ac[cur][u]) * k + vc);
                if (jb + U < m) load_grp(jb + U, m, base_lead, av[cur ^ 1], ac[cur ^ 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool on = jb + u < len && jb + u < m;
#pragma unroll
                    for (int q = 0; q < VPL; ++q) {
                        T &aq = reinterpret_cast<T *>(&acc)[q];
                        const T s = __builtin_fma(av[cur][u], reinterpret_cast<const T *>(&xv[u])[q], aq);
                        aq = on ? s : aq;
                    }
                }
            };
            for (int jb = 0; jb < m; jb += 2 * U) {
                grp(jb, 0);
                if (jb + U < m) grp(jb + U, 1);
            }
        }
        if (i < n_rows && v < k)            // Y is written once: stored non-temporally
            __builtin_nontemporal_store(acc, reinterpret_cast<V *>(Y + int64_t((flags & PJDS_Y_PERMUTED) ? i : perm[i]) * k + v));
    }
}

template <class T, int BR, int LPR, int VPL>
void launch_lv(const pjds_info &in, int64_t tile, int64_t halo, int32_t cap, int32_t k, const int32_t *rl,
               const int64_t *off, const int32_t *cp, const void *vp, const int32_t *perm, const void *X, void *Y,
               uint32_t flags, hipStream_t s) {
    const dim3 grid(unsigned(ceil_div(in.n_pad, tile)), unsigned(ceil_div(k, LPR * VPL)));
    const size_t lds = size_t(std::max(cap, 1)) * LPR * VPL * sizeof(T);
    launch_main((spmmv_xlds_kernel<T, BR, LPR, VPL>), grid, dim3(kThreads), lds, s, in.n_rows, in.n_cols,
                       in.n_pad, in.sort_window, halo, tile, cap, k, rl, off, cp, static_cast<const T *>(vp), perm,
                       static_cast<const T *>(X), static_cast<T *>(Y), flags);
}

template <class T, int BR, int VPL>
void launch_v(const pjds_info &in, int32_t lpr, int64_t tile, int64_t halo, int32_t cap, int32_t k,
              const int32_t *rl, const int64_t *off, const int32_t *cp, const void *vp, const int32_t *perm,
              const void *X, void *Y, uint32_t flags, hipStream_t s) {
    if (lpr == 1) launch_lv<T, BR, 1, VPL>(in, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
    else if (lpr == 2) launch_lv<T, BR, 2, VPL>(in, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
    else launch_lv<T, BR, 4, VPL>(in, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
}

template <class T, int BR>
void launch_br(const pjds_info &in, int32_t vpl, int32_t lpr, int64_t tile, int64_t halo, int32_t cap, int32_t k,
               const int32_t *rl, const int64_t *off, const int32_t *cp, const void *vp, const int32_t *perm,
               const void *X, void *Y, uint32_t flags, hipStream_t s) {
    if (vpl == 1) launch_v<T, BR, 1>(in, lpr, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
    else if (vpl == 2) launch_v<T, BR, 2>(in, lpr, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
    else launch_v<T, BR, 4>(in, lpr, tile, halo, cap, k, rl, off, cp, vp, perm, X, Y, flags, s);
}

}  // namespace
}  // namespace pjds

using namespace pjds;

extern "C" int pjds_spmmv_xlds(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                               const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                               int32_t dtype, int32_t k, int32_t vectors_per_tile, int32_t vectors_per_lane,
                               const void *d_X, void *d_Y, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                               void *stream) {
    if (int rc = check_product_info(info, dtype)) return rc;
    if (flags & ~PJDS_Y_PERMUTED) return fail(PJDS_ERR_ARG, "unknown product flags 0x%x", flags);
    if (info->flags & PJDS_LANES_MASK) return fail(PJDS_ERR_UNSUPPORTED, "SpMMV with several lanes per row");
    const int64_t w = info->sort_window;
    if (!(info->flags & PJDS_LAYOUT_BLOCK) || w >= info->n_rows || w % kWave)
        return fail(PJDS_ERR_ARG, "X staging needs the block layout and a sort window (a multiple of %d)", kWave);
    if (k < 1) return fail(PJDS_ERR_ARG, "k = %d", k);
    const int32_t t = vectors_per_tile, vpl = vectors_per_lane;
    if (vpl != 1 && vpl != 2 && vpl != 4) return fail(PJDS_ERR_ARG, "vectors_per_lane %d: must be 1, 2 or 4", vpl);
    if (k % vpl) return fail(PJDS_ERR_ARG, "k = %d must be a multiple of vectors_per_lane %d", k, vpl);
    const int32_t lpr = t / vpl;
    if (t % vpl || (lpr != 1 && lpr != 2 && lpr != 4))
        return fail(PJDS_ERR_ARG, "vectors_per_tile %d: vectors_per_lane times 1, 2 or 4", t);
    if (x_halo < 0) return fail(PJDS_ERR_ARG, "x_halo %d", x_halo);
    const int64_t tile = tile_rows == 0 ? std::max<int64_t>(w, 1024) : tile_rows;
    if (tile < kWave || tile % kWave) return fail(PJDS_ERR_ARG, "tile_rows %lld: a multiple of %d", (long long)tile, kWave);
    if (ceil_div(k, t) > 65535 || ceil_div(info->n_pad, tile) > INT32_MAX) return fail(PJDS_ERR_ARG, "grid too large");
    if (info->n_rows == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_Y) return fail(PJDS_ERR_ARG, "NULL device array");
    if (info->nnz_stored && (!d_col_p || !d_val_p)) return fail(PJDS_ERR_ARG, "NULL device array");
    // every tile copies its rows of X into LDS, even when the matrix has no entries
    if (info->n_cols && !d_X) return fail(PJDS_ERR_ARG, "d_X is NULL");
    if (!(flags & PJDS_Y_PERMUTED) && !d_perm) return fail(PJDS_ERR_ARG, "d_perm is NULL (needed to scatter Y)");
    const int64_t elt = dtype == PJDS_F64 ? 8 : 4;
    if ((reinterpret_cast<uintptr_t>(d_X) | reinterpret_cast<uintptr_t>(d_Y)) % uintptr_t(elt * vpl))
        return fail(PJDS_ERR_ARG, "X and Y must be aligned to vectors_per_lane values");
    // staged rows per workgroup: what the widest tile needs (its windows plus the halo), cut at
    // the LDS cap; X rows past the cut are read from global memory
    const int64_t need = ceil_div(tile + w - 1, w) * w + 2 * int64_t(x_halo);
    const int32_t cap = int32_t(std::max<int64_t>(1, std::min({need, info->n_cols, kMaxLds / (int64_t(t) * elt)})));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int br = info->block_height;
    auto go = [&](auto tag) {
        using T = decltype(tag);
        if (br == 32) launch_br<T, 32>(*info, vpl, lpr, tile, x_halo, cap, k, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_X, d_Y, flags, s);
        else if (br == 64) launch_br<T, 64>(*info, vpl, lpr, tile, x_halo, cap, k, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_X, d_Y, flags, s);
        else launch_br<T, 128>(*info, vpl, lpr, tile, x_halo, cap, k, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_X, d_Y, flags, s);
    };
    if (dtype == PJDS_F64) go(double{});
    else go(float{});
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PJDS_OK : fail(PJDS_ERR_HIP, "pjds_spmmv_xlds: %s", hipGetErrorString(e));
}
