// Matrix features for the learned configuration tuner (pjds_features).
//
// 24 numbers describing the size, the row-length distribution, the padding the pJDS and
// ELLPACK-R formats would need, and where the non-zeros sit relative to the diagonal.
// Row-length statistics use every row; statistics of the offsets d = col - row use a
// deterministic sample of at most 2^20 entries (every s-th entry, s = ceil(nnz / 2^20)).
// All sums run in binary64 in a fixed order; the result is rounded to float.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace pjds {
namespace {

// sum over blocks of b_r consecutive rows (after a descending sort of the lengths inside
// windows of `window` rows) of b_r times the block maximum
double padded_entries(const std::vector<int64_t> &len, int64_t b_r, int64_t window) {
    const int64_t n = int64_t(len.size());
    double total = 0.0;
    std::vector<int64_t> w;
    for (int64_t w0 = 0; w0 < n; w0 += window) {
        const int64_t w1 = std::min(n, w0 + window);
        w.assign(len.begin() + w0, len.begin() + w1);
        std::sort(w.begin(), w.end(), [](int64_t a, int64_t b) { return a > b; });
        for (size_t r = 0; r < w.size(); r += size_t(b_r)) total += double(b_r) * double(w[r]);
    }
    return total;
}

double quantile_sorted(const std::vector<int64_t> &s, double q) {
    // nearest-rank on the ascending sort: element ceil(q * n) - 1 (at least 0)
    const int64_t n = int64_t(s.size());
    int64_t k = int64_t(std::ceil(q * double(n))) - 1;
    k = std::max<int64_t>(0, std::min(n - 1, k));
    return double(s[size_t(k)]);
}

}  // namespace
}  // namespace pjds

using namespace pjds;

extern "C" int pjds_features(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr,
                             const int32_t *col_idx, float *out) {
    if (!out) return fail(PJDS_ERR_ARG, "out is NULL");
    if (n_rows < 1 || n_cols < 1) return fail(PJDS_ERR_ARG, "features need at least one row and column");
    if (!row_ptr) return fail(PJDS_ERR_ARG, "row_ptr is NULL");
    if (row_ptr[0] != 0) return fail(PJDS_ERR_INDEX, "row_ptr[0] != 0");
    for (int64_t i = 0; i < n_rows; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return fail(PJDS_ERR_INDEX, "row_ptr decreases at row %lld", (long long)i);
    const int64_t nnz = row_ptr[n_rows];
    if (nnz > 0 && !col_idx) return fail(PJDS_ERR_ARG, "col_idx is NULL");
    double f[24];
    std::memset(f, 0, sizeof f);

    std::vector<int64_t> len(static_cast<size_t>(n_rows));
    for (int64_t i = 0; i < n_rows; ++i) len[size_t(i)] = row_ptr[i + 1] - row_ptr[i];
    const double N = double(n_rows), mean = double(nnz) / N;
    double m2 = 0, m3 = 0, m4 = 0;
    int64_t lmin = len[0], lmax = len[0], empty = 0;
    for (int64_t L : len) {
        const double d = double(L) - mean;
        m2 += d * d;
        m3 += d * d * d;
        m4 += d * d * d * d;
        lmin = std::min(lmin, L);
        lmax = std::max(lmax, L);
        empty += L == 0;
    }
    m2 /= N;
    m3 /= N;
    m4 /= N;
    const double sd = std::sqrt(m2);
    std::vector<int64_t> sorted = len;
    std::sort(sorted.begin(), sorted.end());
    f[0] = std::log2(N);
    f[1] = std::log2(double(nnz) + 1.0);
    f[2] = mean;
    f[3] = sd;
    f[4] = sd > 0 ? m3 / (sd * sd * sd) : 0.0;                 // skewness
    f[5] = sd > 0 ? m4 / (m2 * m2) - 3.0 : 0.0;                // excess kurtosis
    f[6] = double(lmin);
    f[7] = std::log2(double(lmax) + 1.0);
    f[8] = mean > 0 ? double(lmax) / mean : 0.0;
    f[9] = double(empty) / N;
    f[10] = mean > 0 ? quantile_sorted(sorted, 0.50) / mean : 0.0;
    f[11] = mean > 0 ? quantile_sorted(sorted, 0.90) / mean : 0.0;
    f[12] = mean > 0 ? quantile_sorted(sorted, 0.99) / mean : 0.0;
    const double nz = std::max<double>(double(nnz), 1.0);
    const double n_pad64 = std::ceil(N / 64.0) * 64.0;
    std::vector<int64_t> padded = len;
    padded.resize(size_t(n_pad64), 0);
    f[13] = std::log2((n_pad64 * double(lmax) + 1.0) / nz);   // ELLPACK-R stored / nnz
    f[14] = padded_entries(padded, 64, int64_t(n_pad64)) / nz;  // pJDS b_r 64, global sort
    f[15] = padded_entries(padded, 64, 4096) / nz;               // pJDS b_r 64, window 4096

    // offsets d = col - row on a deterministic sample of the entries
    const int64_t cap = int64_t(1) << 20;
    const int64_t step = nnz > cap ? (nnz + cap - 1) / cap : 1;
    double sum_a = 0, sum_a2 = 0;
    int64_t n_s = 0, near64 = 0, near4k = 0, maxabs = 0;
    std::unordered_map<int64_t, int64_t> diag;
    int64_t row = 0;
    for (int64_t k = 0; k < nnz; k += step) {
        while (row_ptr[row + 1] <= k) ++row;
        const int64_t d = int64_t(col_idx[k]) - row;
        const int64_t a = d < 0 ? -d : d;
        sum_a += double(a);
        sum_a2 += double(a) * double(a);
        near64 += a <= 64;
        near4k += a <= 4096;
        maxabs = std::max(maxabs, a);
        ++diag[d];
        ++n_s;
    }
    if (n_s > 0) {
        const double ns = double(n_s), scale = double(std::max(n_rows, n_cols));
        const double ma = sum_a / ns;
        f[16] = double(maxabs) / scale;
        f[17] = ma / scale;
        f[18] = std::sqrt(std::max(0.0, sum_a2 / ns - ma * ma)) / scale;
        f[19] = double(near64) / ns;
        f[20] = double(near4k) / ns;
        f[21] = std::log(double(diag.size()) / ns);
        std::vector<int64_t> counts;
        counts.reserve(diag.size());
        for (auto &kv : diag) counts.push_back(kv.second);
        std::sort(counts.begin(), counts.end(), [](int64_t a, int64_t b) { return a > b; });
        int64_t top = 0;
        for (size_t q = 0; q < counts.size() && q < 16; ++q) top += counts[q];
        f[22] = double(top) / ns;
    }
    // x-line reuse: for up to 256 evenly spaced blocks of 64 consecutive rows, entries per
    // distinct 16-element column segment (a 128-byte line of binary64 x), averaged
    {
        const int64_t blocks = (n_rows + 63) / 64;
        const int64_t nb = std::min<int64_t>(blocks, 256);
        double acc = 0;
        int64_t used = 0;
        std::vector<int64_t> lines;
        for (int64_t q = 0; q < nb; ++q) {
            const int64_t b = q * blocks / nb;
            const int64_t r0 = b * 64, r1 = std::min(n_rows, r0 + 64);
            lines.clear();
            for (int64_t k = row_ptr[r0]; k < row_ptr[r1]; ++k) lines.push_back(int64_t(col_idx[k]) >> 4);
            if (lines.empty()) continue;
            const double e = double(lines.size());
            std::sort(lines.begin(), lines.end());
            const double distinct = double(std::unique(lines.begin(), lines.end()) - lines.begin());
            acc += e / distinct;
            ++used;
        }
        f[23] = used ? acc / double(used) : 0.0;
    }
    for (int q = 0; q < 24; ++q) out[q] = float(f[q]);
    return PJDS_OK;
}
