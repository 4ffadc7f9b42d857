// Host-side CSR -> pJDS and CSR -> ELLPACK-R conversion (Sect. 2.1 of Kreutzer et al.,
// arXiv:1112.5588: the "sort" and "pad" steps, col_start[] of Listing 2, and the
// column-major ELLPACK-R storage of Listing 1).
//
// The sort is a stable counting sort by row length (descending) inside each sort window,
// O(rows + longest row) per window.  The fill walks one block at a time, so each block's
// b_r x M_b tile (or its slice of every jagged diagonal in the JD layout) is written with
// unit stride; blocks are distributed over host threads and write disjoint ranges, so the
// result does not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace pjds {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
}

const char *get_error() { return g_error.c_str(); }

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int host_threads() {
    if (const char *s = std::getenv("PJDS_NUM_THREADS")) {
        int v = std::atoi(s);
        if (v >= 1) return v > 256 ? 256 : v;
    }
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 1;
    return h > 32 ? 32 : int(h);
}

namespace {

constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;

// row_ptr checks shared by every planner: starts at 0, never decreases, row lengths and
// row counts fit the int32 index types.
int check_row_ptr(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr) {
    if (n_rows < 0 || n_cols < 0) return fail(PJDS_ERR_ARG, "negative size (n_rows=%lld, n_cols=%lld)", (long long)n_rows, (long long)n_cols);
    if (n_rows > kMaxIndex || n_cols > kMaxIndex)
        return fail(PJDS_ERR_OVERFLOW, "n_rows and n_cols must be below 2^31");
    if (!row_ptr) return fail(PJDS_ERR_ARG, "row_ptr is NULL");
    if (row_ptr[0] != 0) return fail(PJDS_ERR_INDEX, "row_ptr[0] = %lld, expected 0", (long long)row_ptr[0]);
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t len = row_ptr[i + 1] - row_ptr[i];
        if (len < 0) return fail(PJDS_ERR_INDEX, "row_ptr decreases at row %lld", (long long)i);
        if (len > kMaxIndex) return fail(PJDS_ERR_OVERFLOW, "row %lld is longer than 2^31-1", (long long)i);
    }
    return PJDS_OK;
}

int check_columns(int64_t nnz, int64_t n_cols, const int32_t *col) {
    if (nnz > 0 && !col) return fail(PJDS_ERR_ARG, "col_idx is NULL");
    std::atomic<int64_t> bad{-1};
    parallel_ranges(nnz, [&](int, int64_t b, int64_t e) {
        for (int64_t k = b; k < e; ++k)
            if (col[k] < 0 || col[k] >= n_cols) {
                int64_t expect = -1;
                bad.compare_exchange_strong(expect, k);
                return;
            }
    });
    if (bad.load() >= 0)
        return fail(PJDS_ERR_INDEX, "column index %d at entry %lld outside [0, %lld)",
                    col[bad.load()], (long long)bad.load(), (long long)n_cols);
    return PJDS_OK;
}

// Stable counting sort by row length, longest first, inside windows of `window` rows.
// perm[new] = old; row_len[new] = length (row_len sized n_pad, tail zero-filled).
void sort_rows(int64_t n_rows, int64_t n_pad, int64_t window, const int64_t *row_ptr,
               int32_t *perm, int32_t *row_len) {
    int64_t n_win = n_rows > 0 ? ceil_div(n_rows, window) : 0;
    auto one_window = [&](int64_t w, std::vector<int64_t> &count) {
        int64_t w0 = w * window, w1 = std::min(n_rows, w0 + window);
        int64_t lmax = 0;
        for (int64_t i = w0; i < w1; ++i) lmax = std::max(lmax, row_ptr[i + 1] - row_ptr[i]);
        count.assign(size_t(lmax) + 2, 0);
        for (int64_t i = w0; i < w1; ++i) ++count[size_t(row_ptr[i + 1] - row_ptr[i])];
        // first slot of length L in descending order = rows strictly longer than L
        int64_t run = 0;
        for (int64_t L = lmax; L >= 0; --L) {
            int64_t c = count[size_t(L)];
            count[size_t(L)] = run;
            run += c;
        }
        for (int64_t i = w0; i < w1; ++i) {
            int64_t L = row_ptr[i + 1] - row_ptr[i];
            int64_t dst = w0 + count[size_t(L)]++;
            perm[dst] = int32_t(i);
            row_len[dst] = int32_t(L);
        }
    };
    parallel_ranges(n_win < 65536 && n_rows >= 65536 ? n_win * 65536 : n_win, [&](int, int64_t b, int64_t e) {
        // when there are few windows, the range is scaled so that threads still split them
        int64_t scale = (n_win < 65536 && n_rows >= 65536) ? 65536 : 1;
        std::vector<int64_t> count;
        for (int64_t w = ceil_div(b, scale); w * scale < e && w < n_win; ++w) one_window(w, count);
    });
    for (int64_t i = n_rows; i < n_pad; ++i) row_len[i] = 0;
}

// T = 2^k lanes per row from the conversion flags (1 without PJDS_LANES).
inline int32_t lanes_per_row(uint32_t flags) { return int32_t(1) << ((flags & PJDS_LANES_MASK) >> PJDS_LANES_SHIFT); }

struct Plan {
    int64_t n_pad = 0, n_blocks = 0, nnz_stored = 0, n_chunks = 0, n_split = 0;
    int32_t max_len = 0;
    std::vector<int64_t> block_max;
};

// Block maxima, stored entries (b_r * T * ceil(M_b / T) per block) and the long-row work
// items of wave groups longer than split_len.
void size_blocks(int64_t n_pad, int32_t b_r, int32_t lanes, int32_t split_len, const int32_t *row_len, Plan &p) {
    p.n_pad = n_pad;
    p.n_blocks = n_pad / b_r;
    p.block_max.assign(size_t(p.n_blocks), 0);
    int64_t stored = 0;
    int32_t mx = 0;
    for (int64_t b = 0; b < p.n_blocks; ++b) {
        int32_t m = 0;
        for (int32_t r = 0; r < b_r; ++r) m = std::max(m, row_len[b * b_r + r]);
        p.block_max[size_t(b)] = m;
        stored += int64_t(b_r) * lanes * ceil_div(m, lanes);
        mx = std::max(mx, m);
    }
    p.nnz_stored = stored;
    p.max_len = mx;
    p.n_chunks = p.n_split = 0;
    if (split_len > 0) {
        int64_t groups = ceil_div(n_pad, kWave);
        for (int64_t g = 0; g < groups; ++g) {
            int32_t m = 0;
            for (int64_t i = g * kWave; i < std::min(n_pad, (g + 1) * kWave); ++i) m = std::max(m, row_len[i]);
            if (m > split_len) {
                p.n_chunks += ceil_div(m, split_len);
                ++p.n_split;
            }
        }
    }
}

int plan_common(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, int32_t b_r,
                int64_t sort_window, uint32_t flags, int32_t split_len, int64_t &window,
                int32_t &split) {
    if (int rc = check_row_ptr(n_rows, n_cols, row_ptr)) return rc;
    if (flags & ~(PJDS_LAYOUT_BLOCK | PJDS_SYMMETRIC | PJDS_LANES_MASK))
        return fail(PJDS_ERR_ARG, "unknown conversion flags 0x%x", flags);
    const int32_t lanes = lanes_per_row(flags);
    if (lanes > kWave) return fail(PJDS_ERR_ARG, "PJDS_LANES(k) needs k <= 6");
    if (lanes > 1) {
        if (!(flags & PJDS_LAYOUT_BLOCK)) return fail(PJDS_ERR_ARG, "PJDS_LANES needs PJDS_LAYOUT_BLOCK");
        if (b_r != kWave / lanes)
            return fail(PJDS_ERR_ARG, "block_height %d: with %d lanes per row it must be %d", b_r, lanes, kWave / lanes);
    } else if (b_r != 32 && b_r != 64 && b_r != 128) {
        return fail(PJDS_ERR_ARG, "block_height %d: must be 32, 64 or 128", b_r);
    }
    if ((flags & PJDS_SYMMETRIC) && n_rows != n_cols)
        return fail(PJDS_ERR_ARG, "PJDS_SYMMETRIC needs a square matrix (%lld x %lld)", (long long)n_rows, (long long)n_cols);
    if (sort_window <= 0 || sort_window >= n_rows) {
        window = n_rows > 0 ? n_rows : 1;
    } else {
        int64_t unit = std::max<int64_t>(kWave, b_r);
        if (sort_window % unit)
            return fail(PJDS_ERR_ARG, "sort_window %lld must be a multiple of %lld", (long long)sort_window, (long long)unit);
        if (!(flags & PJDS_LAYOUT_BLOCK))
            return fail(PJDS_ERR_ARG, "the JD layout needs a global sort; use PJDS_LAYOUT_BLOCK with a sort window");
        window = sort_window;
    }
    if (split_len < 0 || lanes > 1) split = 0;
    else if (split_len == 0) split = 128;
    else if (split_len % 8) return fail(PJDS_ERR_ARG, "split_len %d must be a multiple of 8", split_len);
    else split = split_len;
    int64_t n_pad = ceil_div(n_rows, b_r) * b_r;
    if (n_pad > kMaxIndex) return fail(PJDS_ERR_OVERFLOW, "padded row count exceeds 2^31-1");
    return PJDS_OK;
}

template <class T>
void fill_blocks(const pjds_info &in, const int64_t *row_ptr, const int32_t *col, const T *val,
                 const int32_t *perm, const int32_t *row_len, const int64_t *offsets,
                 const int32_t *invperm, int32_t *col_p, T *val_p, const std::vector<int64_t> &bmax) {
    const int32_t b_r = in.block_height, lanes = lanes_per_row(in.flags);
    const bool jd = !(in.flags & PJDS_LAYOUT_BLOCK);
    const int64_t n = in.n_rows;
    if (lanes > 1) {
        // T lanes per row: step q of block b is the 64-slot segment at offsets[b] + 64 q,
        // slot r * T + t of it holds entry j = q * T + t of the block's row r
        parallel_ranges(in.n_blocks, [&](int, int64_t b0, int64_t b1) {
            for (int64_t b = b0; b < b1; ++b) {
                const int64_t W = ceil_div(bmax[size_t(b)], lanes);
                for (int64_t q = 0; q < W; ++q)
                    for (int32_t r = 0; r < b_r; ++r)
                        for (int32_t t = 0; t < lanes; ++t) {
                            const int64_t i = b * b_r + r, j = q * lanes + t;
                            const int64_t a = offsets[b] + q * kWave + r * lanes + t;
                            if (i < n && j < row_len[i]) {
                                const int64_t k = row_ptr[perm[i]] + j;
                                const int32_t c = col[k];
                                col_p[a] = invperm ? invperm[c] : c;
                                val_p[a] = val[k];
                            } else {
                                col_p[a] = 0;
                                val_p[a] = T(0);
                            }
                        }
            }
        });
        return;
    }
    parallel_ranges(in.n_blocks, [&](int, int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t M = bmax[size_t(b)];
            for (int64_t j = 0; j < M; ++j) {
                const int64_t base = jd ? offsets[j] + b * b_r : offsets[b] + j * b_r;
                for (int32_t r = 0; r < b_r; ++r) {
                    const int64_t i = b * b_r + r;
                    const int64_t a = base + r;
                    if (i < n && j < row_len[i]) {
                        const int64_t k = row_ptr[perm[i]] + j;
                        const int32_t c = col[k];
                        col_p[a] = invperm ? invperm[c] : c;
                        val_p[a] = val[k];
                    } else {
                        col_p[a] = 0;
                        val_p[a] = T(0);
                    }
                }
            }
        }
    });
}

}  // namespace
}  // namespace pjds

using namespace pjds;

extern "C" {

const char *pjds_last_error(void) { return get_error(); }
const char *pjds_version(void) { return "libpjds 0.1 (gfx950)"; }

int pjds_plan(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, int32_t block_height,
              int64_t sort_window, uint32_t flags, int32_t split_len, pjds_info *out) {
    if (!out) return fail(PJDS_ERR_ARG, "out is NULL");
    int64_t window;
    int32_t split;
    if (int rc = plan_common(n_rows, n_cols, row_ptr, block_height, sort_window, flags, split_len, window, split)) return rc;
    const int64_t n_pad = ceil_div(n_rows, block_height) * block_height;
    std::vector<int32_t> perm, row_len;
    try {
        perm.resize(size_t(std::max<int64_t>(n_rows, 1)));
        row_len.resize(size_t(std::max<int64_t>(n_pad, 1)));
    } catch (const std::bad_alloc &) {
        return fail(PJDS_ERR_NOMEM, "host allocation of %lld rows failed", (long long)n_pad);
    }
    sort_rows(n_rows, n_pad, window, row_ptr, perm.data(), row_len.data());
    Plan p;
    size_blocks(n_pad, block_height, lanes_per_row(flags), split, row_len.data(), p);
    pjds_info info{};
    info.n_rows = n_rows;
    info.n_cols = n_cols;
    info.n_pad = n_pad;
    info.n_blocks = p.n_blocks;
    info.nnz = row_ptr[n_rows];
    info.nnz_stored = p.nnz_stored;
    info.sort_window = window;
    info.n_offsets = (flags & PJDS_LAYOUT_BLOCK) ? p.n_blocks + 1 : int64_t(p.max_len) + 1;
    info.block_height = block_height;
    info.max_row_len = p.max_len;
    info.flags = flags;
    info.split_len = split;
    info.n_chunks = p.n_chunks;
    info.n_split_groups = p.n_split;
    *out = info;
    return PJDS_OK;
}

int pjds_convert(const pjds_info *info, const int64_t *row_ptr, const int32_t *col_idx,
                 const void *val, int32_t dtype, int32_t *perm, int32_t *row_len,
                 int64_t *offsets, int32_t *col_p, void *val_p, int32_t *sched) {
    if (!info) return fail(PJDS_ERR_ARG, "info is NULL");
    const pjds_info in = *info;
    int64_t window;
    int32_t split;
    if (int rc = plan_common(in.n_rows, in.n_cols, row_ptr, in.block_height,
                             in.sort_window >= in.n_rows ? 0 : in.sort_window, in.flags,
                             in.split_len == 0 ? -1 : in.split_len, window, split))
        return rc;
    if (row_ptr[in.n_rows] != in.nnz) return fail(PJDS_ERR_ARG, "info does not match row_ptr (nnz %lld vs %lld)", (long long)in.nnz, (long long)row_ptr[in.n_rows]);
    // every size the caller sized its buffers by must be the planner's own, before anything is
    // allocated from it or written
    if (in.n_pad != ceil_div(in.n_rows, in.block_height) * in.block_height || in.n_blocks != in.n_pad / in.block_height ||
        in.sort_window != window || in.split_len != split)
        return fail(PJDS_ERR_ARG, "info does not match the planner's sizes (re-run pjds_plan)");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    if ((in.n_rows && !perm) || !row_len || !offsets) return fail(PJDS_ERR_ARG, "NULL output array");
    if (in.nnz_stored && (!col_p || !val_p)) return fail(PJDS_ERR_ARG, "NULL output array");
    if (in.nnz && !val) return fail(PJDS_ERR_ARG, "val is NULL");
    if (in.n_chunks && !sched) return fail(PJDS_ERR_ARG, "sched is NULL but %lld work items are planned", (long long)in.n_chunks);
    if (int rc = check_columns(in.nnz, in.n_cols, col_idx)) return rc;

    // Sort into temporaries first, verify the plan still matches, then write outputs.
    std::vector<int32_t> tperm, tlen;
    try {
        tperm.resize(size_t(std::max<int64_t>(in.n_rows, 1)));
        tlen.resize(size_t(std::max<int64_t>(in.n_pad, 1)));
    } catch (const std::bad_alloc &) {
        return fail(PJDS_ERR_NOMEM, "host allocation failed");
    }
    sort_rows(in.n_rows, in.n_pad, window, row_ptr, tperm.data(), tlen.data());
    Plan p;
    size_blocks(in.n_pad, in.block_height, lanes_per_row(in.flags), in.split_len, tlen.data(), p);
    const int64_t n_offsets = (in.flags & PJDS_LAYOUT_BLOCK) ? p.n_blocks + 1 : int64_t(p.max_len) + 1;
    if (p.nnz_stored != in.nnz_stored || p.n_chunks != in.n_chunks || p.n_split != in.n_split_groups ||
        p.max_len != in.max_row_len || n_offsets != in.n_offsets)
        return fail(PJDS_ERR_ARG, "info does not match the matrix (re-run pjds_plan)");

    std::vector<int32_t> invperm;
    if (in.flags & PJDS_SYMMETRIC) {
        invperm.resize(size_t(std::max<int64_t>(in.n_rows, 1)));
        for (int64_t i = 0; i < in.n_rows; ++i) invperm[size_t(tperm[size_t(i)])] = int32_t(i);
    }
    if (in.n_rows) std::memcpy(perm, tperm.data(), sizeof(int32_t) * size_t(in.n_rows));
    std::memcpy(row_len, tlen.data(), sizeof(int32_t) * size_t(in.n_pad));
    const int32_t b_r = in.block_height, lanes = lanes_per_row(in.flags);
    if (in.flags & PJDS_LAYOUT_BLOCK) {
        offsets[0] = 0;
        for (int64_t b = 0; b < p.n_blocks; ++b)
            offsets[b + 1] = offsets[b] + int64_t(b_r) * lanes * ceil_div(p.block_max[size_t(b)], lanes);
    } else {
        // col_start[j+1] - col_start[j] = b_r * #{blocks with M_b > j}; with a global sort
        // the block maxima do not increase, so count blocks per maximum and sweep j upward.
        std::vector<int64_t> per_max(size_t(p.max_len) + 1, 0);
        for (int64_t b = 0; b < p.n_blocks; ++b) ++per_max[size_t(p.block_max[size_t(b)])];
        int64_t longer = p.n_blocks - per_max[0];  // blocks with M_b > 0
        offsets[0] = 0;
        for (int64_t j = 0; j < p.max_len; ++j) {
            offsets[j + 1] = offsets[j] + int64_t(b_r) * longer;
            longer -= per_max[size_t(j) + 1];      // blocks with M_b == j+1 end here
        }
    }
    const int32_t *ip = invperm.empty() ? nullptr : invperm.data();
    if (dtype == PJDS_F64)
        fill_blocks<double>(in, row_ptr, col_idx, static_cast<const double *>(val), tperm.data(),
                            tlen.data(), offsets, ip, col_p, static_cast<double *>(val_p), p.block_max);
    else
        fill_blocks<float>(in, row_ptr, col_idx, static_cast<const float *>(val), tperm.data(),
                           tlen.data(), offsets, ip, col_p, static_cast<float *>(val_p), p.block_max);
    // Long-row work items: (wave group, chunk index, chunks in group, first item of group).
    if (in.n_chunks) {
        int64_t groups = ceil_div(in.n_pad, kWave), w = 0;
        for (int64_t g = 0; g < groups; ++g) {
            int32_t m = 0;
            for (int64_t i = g * kWave; i < std::min(in.n_pad, (g + 1) * kWave); ++i) m = std::max(m, tlen[size_t(i)]);
            if (m <= in.split_len) continue;
            int32_t nc = int32_t(ceil_div(m, in.split_len));
            int64_t first = w;
            for (int32_t c = 0; c < nc; ++c, ++w) {
                sched[4 * w + 0] = int32_t(g);
                sched[4 * w + 1] = c;
                sched[4 * w + 2] = nc;
                sched[4 * w + 3] = int32_t(first);
            }
        }
    }
    return PJDS_OK;
}

int pjds_split_count(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, const int32_t *col_idx,
                     int64_t c0, int64_t c1, int64_t *nnz_local) {
    if (!nnz_local) return fail(PJDS_ERR_ARG, "nnz_local is NULL");
    if (int rc = check_row_ptr(n_rows, n_cols, row_ptr)) return rc;
    if (c0 < 0 || c1 < c0 || c1 > n_cols) return fail(PJDS_ERR_ARG, "column range [%lld, %lld) outside [0, %lld]",
                                                     (long long)c0, (long long)c1, (long long)n_cols);
    const int64_t nnz = row_ptr[n_rows];
    if (int rc = check_columns(nnz, n_cols, col_idx)) return rc;
    int64_t loc = 0;
    for (int64_t k = 0; k < nnz; ++k) loc += col_idx[k] >= c0 && col_idx[k] < c1;
    *nnz_local = loc;
    return PJDS_OK;
}

int pjds_split_columns(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, const int32_t *col_idx,
                       const void *val, int32_t dtype, int64_t c0, int64_t c1, int64_t *rp_loc,
                       int32_t *col_loc, void *val_loc, int64_t *rp_nl, int32_t *col_nl, void *val_nl) {
    int64_t loc = 0;
    if (int rc = pjds_split_count(n_rows, n_cols, row_ptr, col_idx, c0, c1, &loc)) return rc;
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    const int64_t nnz = row_ptr[n_rows];
    if (!rp_loc || !rp_nl) return fail(PJDS_ERR_ARG, "NULL row pointer output");
    if ((loc && (!col_loc || !val_loc)) || (nnz - loc && (!col_nl || !val_nl)) || (nnz && !val))
        return fail(PJDS_ERR_ARG, "NULL array");
    const size_t esz = dtype == PJDS_F64 ? 8 : 4;
    const char *v = static_cast<const char *>(val);
    char *vl = static_cast<char *>(val_loc), *vn = static_cast<char *>(val_nl);
    int64_t a = 0, b = 0;
    rp_loc[0] = rp_nl[0] = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col_idx[k] >= c0 && col_idx[k] < c1) {
                col_loc[a] = col_idx[k];
                std::memcpy(vl + size_t(a) * esz, v + size_t(k) * esz, esz);
                ++a;
            } else {
                col_nl[b] = col_idx[k];
                std::memcpy(vn + size_t(b) * esz, v + size_t(k) * esz, esz);
                ++b;
            }
        }
        rp_loc[i + 1] = a;
        rp_nl[i + 1] = b;
    }
    return PJDS_OK;
}

int ellr_plan(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, pjds_info *out) {
    if (!out) return fail(PJDS_ERR_ARG, "out is NULL");
    if (int rc = check_row_ptr(n_rows, n_cols, row_ptr)) return rc;
    int64_t n_pad = ceil_div(n_rows, kWave) * kWave;
    int64_t mx = 0;
    for (int64_t i = 0; i < n_rows; ++i) mx = std::max(mx, row_ptr[i + 1] - row_ptr[i]);
    if (mx > 0 && n_pad > INT64_MAX / mx) return fail(PJDS_ERR_OVERFLOW, "ELLPACK-R size overflows int64");
    pjds_info info{};
    info.n_rows = n_rows;
    info.n_cols = n_cols;
    info.n_pad = n_pad;
    info.n_blocks = n_pad / kWave;
    info.nnz = row_ptr[n_rows];
    info.nnz_stored = n_pad * mx;
    info.sort_window = 0;
    info.n_offsets = 0;
    info.block_height = kWave;
    info.max_row_len = int32_t(mx);
    info.flags = 0;
    *out = info;
    return PJDS_OK;
}

int ellr_convert(const pjds_info *info, const int64_t *row_ptr, const int32_t *col_idx,
                 const void *val, int32_t dtype, int32_t *rowmax, int32_t *col_e, void *val_e) {
    if (!info) return fail(PJDS_ERR_ARG, "info is NULL");
    const pjds_info in = *info;
    if (int rc = check_row_ptr(in.n_rows, in.n_cols, row_ptr)) return rc;
    if (row_ptr[in.n_rows] != in.nnz || in.n_pad != ceil_div(in.n_rows, kWave) * kWave)
        return fail(PJDS_ERR_ARG, "info does not match row_ptr");
    if (dtype != PJDS_F64 && dtype != PJDS_F32) return fail(PJDS_ERR_ARG, "dtype %d", dtype);
    if (!rowmax || (in.nnz_stored && (!col_e || !val_e)) || (in.nnz && !val))
        return fail(PJDS_ERR_ARG, "NULL array");
    if (int rc = check_columns(in.nnz, in.n_cols, col_idx)) return rc;
    int64_t mx = 0;
    for (int64_t i = 0; i < in.n_rows; ++i) mx = std::max(mx, row_ptr[i + 1] - row_ptr[i]);
    if (in.max_row_len != mx || in.nnz_stored != in.n_pad * mx)
        return fail(PJDS_ERR_ARG, "info does not match the matrix (re-run ellr_plan)");
    const int64_t n = in.n_rows, np = in.n_pad, L = in.max_row_len;
    auto fill = [&](auto *dst, const auto *src) {
        using T = std::remove_pointer_t<decltype(dst)>;
        parallel_ranges(ceil_div(np, kWave), [&](int, int64_t g0, int64_t g1) {
            for (int64_t g = g0; g < g1; ++g)
                for (int64_t j = 0; j < L; ++j)
                    for (int64_t i = g * kWave; i < (g + 1) * kWave; ++i) {
                        const int64_t a = j * np + i;
                        if (i < n && j < row_ptr[i + 1] - row_ptr[i]) {
                            col_e[a] = col_idx[row_ptr[i] + j];
                            dst[a] = src[row_ptr[i] + j];
                        } else {
                            col_e[a] = 0;
                            dst[a] = T(0);
                        }
                    }
        });
    };
    for (int64_t i = 0; i < np; ++i) rowmax[i] = i < n ? int32_t(row_ptr[i + 1] - row_ptr[i]) : 0;
    if (dtype == PJDS_F64) fill(static_cast<double *>(val_e), static_cast<const double *>(val));
    else fill(static_cast<float *>(val_e), static_cast<const float *>(val));
    return PJDS_OK;
}

}  // extern "C"
