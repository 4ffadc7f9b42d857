// Host conversion code of libpjds under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built with g++ from convert.cpp and features.cpp only (no device code), this program runs
// the planning, conversion, column split, ELLPACK-R and feature entry points on seeded random
// matrices with ragged shapes (empty rows, rows longer than a block, a row count that is not a
// multiple of the block height, one-row and one-column matrices) and on invalid input, and
// checks the invariants of the format that need no reference arithmetic: perm is a bijection,
// the lengths add up to nnz, every padding slot holds value 0 and column 0, every stored
// column is in range, and a refused call leaves its outputs untouched.  A sanitizer report or
// a failed check ends the program with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pjds.h"

namespace {

int failures = 0;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

// SplitMix64 (Steele, Lea, Flood 2014): the driver's own seeded stream.
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int64_t below(int64_t n) { return n > 0 ? int64_t(next() % uint64_t(n)) : 0; }
};

struct Csr {
    int64_t n_rows, n_cols;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> val;
};

Csr random_csr(Rng &r, int64_t n_rows, int64_t n_cols, int max_len, int long_rows) {
    Csr a{n_rows, n_cols, std::vector<int64_t>(size_t(n_rows) + 1, 0), {}, {}};
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t len = r.below(max_len + 1);
        if (r.below(5) == 0) len = 0;                               // empty rows
        if (long_rows && r.below(200) == 0) len = 200 + r.below(600);  // rows over a block
        if (n_cols == 0) len = 0;
        for (int64_t j = 0; j < len; ++j) {
            a.col.push_back(int32_t(r.below(n_cols)));
            a.val.push_back(double(r.below(2001) - 1000) / 7.0);
        }
        a.rp[size_t(i) + 1] = int64_t(a.col.size());
    }
    return a;
}

void check_pjds(const Csr &a, int32_t b_r, int64_t window, uint32_t flags, int32_t split) {
    pjds_info info;
    int rc = pjds_plan(a.n_rows, a.n_cols, a.rp.data(), b_r, window, flags, split, &info);
    if (rc != PJDS_OK) return;                                   // refused plans are tested below
    std::vector<int32_t> perm(size_t(std::max<int64_t>(info.n_rows, 1)));
    std::vector<int32_t> row_len(size_t(std::max<int64_t>(info.n_pad, 1)));
    std::vector<int64_t> offsets(size_t(std::max<int64_t>(info.n_offsets, 1)));
    std::vector<int32_t> col_p(size_t(std::max<int64_t>(info.nnz_stored, 1)), -7);
    std::vector<double> val_p(size_t(std::max<int64_t>(info.nnz_stored, 1)), -7.0);
    std::vector<int32_t> sched(size_t(std::max<int64_t>(4 * info.n_chunks, 1)));
    rc = pjds_convert(&info, a.rp.data(), a.col.data(), a.val.data(), PJDS_F64, perm.data(), row_len.data(),
                      offsets.data(), col_p.data(), val_p.data(), info.n_chunks ? sched.data() : nullptr);
    CHECK(rc == PJDS_OK);
    if (rc != PJDS_OK) return;
    std::vector<char> seen(size_t(info.n_rows), 0);
    int64_t total = 0;
    for (int64_t i = 0; i < info.n_rows; ++i) {
        CHECK(perm[i] >= 0 && perm[i] < info.n_rows);
        if (perm[i] >= 0 && perm[i] < info.n_rows) {
            CHECK(!seen[perm[i]]);
            seen[perm[i]] = 1;
            CHECK(row_len[i] == a.rp[perm[i] + 1] - a.rp[perm[i]]);
        }
        total += row_len[i];
    }
    for (int64_t i = info.n_rows; i < info.n_pad; ++i) CHECK(row_len[i] == 0);
    CHECK(total == info.nnz);
    int64_t zeros = 0;
    for (int64_t k = 0; k < info.nnz_stored; ++k) {
        CHECK(col_p[k] >= 0 && col_p[k] < std::max<int64_t>(a.n_cols, 1));
        if (val_p[k] == 0.0 && col_p[k] == 0) ++zeros;
    }
    CHECK(zeros >= info.nnz_stored - info.nnz);                  // padding is value 0, column 0
    float feats[24];
    if (a.n_rows > 0) CHECK(pjds_features(a.n_rows, a.n_cols, a.rp.data(), a.col.data(), feats) == PJDS_OK);
}

void check_split_and_ellr(const Csr &a, Rng &r) {
    const int64_t c0 = r.below(a.n_cols + 1), c1 = c0 + r.below(a.n_cols - c0 + 1);
    int64_t nl = -1;
    if (pjds_split_count(a.n_rows, a.n_cols, a.rp.data(), a.col.data(), c0, c1, &nl) == PJDS_OK) {
        const int64_t nnz = int64_t(a.col.size());
        CHECK(nl >= 0 && nl <= nnz);
        std::vector<int64_t> rpl(size_t(a.n_rows) + 1), rpn(size_t(a.n_rows) + 1);
        std::vector<int32_t> cl(size_t(std::max<int64_t>(nl, 1))), cn(size_t(std::max<int64_t>(nnz - nl, 1)));
        std::vector<double> vl(cl.size()), vn(cn.size());
        CHECK(pjds_split_columns(a.n_rows, a.n_cols, a.rp.data(), a.col.data(), a.val.data(), PJDS_F64, c0, c1,
                                 rpl.data(), cl.data(), vl.data(), rpn.data(), cn.data(), vn.data()) == PJDS_OK);
        CHECK(rpl[a.n_rows] == nl && rpn[a.n_rows] == nnz - nl);
    }
    pjds_info e;
    if (ellr_plan(a.n_rows, a.n_cols, a.rp.data(), &e) == PJDS_OK && e.nnz_stored < (int64_t(1) << 24)) {
        std::vector<int32_t> rowmax(size_t(std::max<int64_t>(e.n_pad, 1))), ce(size_t(std::max<int64_t>(e.nnz_stored, 1)));
        std::vector<double> ve(ce.size());
        CHECK(ellr_convert(&e, a.rp.data(), a.col.data(), a.val.data(), PJDS_F64, rowmax.data(), ce.data(),
                           ve.data()) == PJDS_OK);
    }
}

void check_refusals(Rng &r) {
    Csr a = random_csr(r, 300, 200, 9, 0);
    pjds_info info;
    // a column out of range is refused before any output is written
    CHECK(pjds_plan(a.n_rows, a.n_cols, a.rp.data(), 64, 0, PJDS_LAYOUT_JD, 0, &info) == PJDS_OK);
    if (!a.col.empty()) a.col[a.col.size() / 2] = int32_t(a.n_cols);
    std::vector<int32_t> perm(size_t(info.n_rows), -3), row_len(size_t(info.n_pad), -3);
    std::vector<int64_t> off(size_t(std::max<int64_t>(info.n_offsets, 1)), -3);
    std::vector<int32_t> col_p(size_t(std::max<int64_t>(info.nnz_stored, 1)), -3);
    std::vector<double> val_p(col_p.size(), -3.0);
    if (!a.col.empty()) {
        CHECK(pjds_convert(&info, a.rp.data(), a.col.data(), a.val.data(), PJDS_F64, perm.data(), row_len.data(),
                           off.data(), col_p.data(), val_p.data(), nullptr) == PJDS_ERR_INDEX);
        for (int32_t p : perm) CHECK(p == -3);
    }
    // an inconsistent plan is refused before any buffer sized from it is written
    pjds_info bad = info;
    bad.n_pad = info.n_pad - 64;
    CHECK(pjds_convert(&bad, a.rp.data(), a.col.data(), a.val.data(), PJDS_F64, perm.data(), row_len.data(),
                       off.data(), col_p.data(), val_p.data(), nullptr) != PJDS_OK);
    // non-monotone row pointers, bad block heights, windows and sizes
    std::vector<int64_t> rp = a.rp;
    rp[5] = rp[6] + 1;
    CHECK(pjds_plan(a.n_rows, a.n_cols, rp.data(), 64, 0, 0, 0, &info) == PJDS_ERR_INDEX);
    CHECK(pjds_plan(a.n_rows, a.n_cols, a.rp.data(), 48, 0, 0, 0, &info) == PJDS_ERR_ARG);
    CHECK(pjds_plan(a.n_rows, a.n_cols, a.rp.data(), 64, 100, PJDS_LAYOUT_BLOCK, 0, &info) == PJDS_ERR_ARG);
    CHECK(pjds_plan(-1, a.n_cols, a.rp.data(), 64, 0, 0, 0, &info) == PJDS_ERR_ARG);
    CHECK(pjds_plan(a.n_rows, a.n_cols, nullptr, 64, 0, 0, 0, &info) != PJDS_OK);
    CHECK(pjds_last_error() != nullptr && std::strlen(pjds_last_error()) > 0);
}

}  // namespace

int main() {
    Rng r{12345};
    const int64_t shapes[][2] = {{0, 0}, {1, 1}, {1, 700}, {63, 63}, {64, 64}, {65, 300}, {257, 257},
                                 {1000, 1}, {3001, 2500}, {4096, 4096}, {9001, 7000}};
    for (auto &sh : shapes) {
        for (int rep = 0; rep < 3; ++rep) {
            Csr a = random_csr(r, sh[0], sh[1], 1 + int(r.below(40)), rep == 2);
            for (int32_t b_r : {32, 64, 128})
                for (uint32_t lay : {PJDS_LAYOUT_JD, PJDS_LAYOUT_BLOCK}) {
                    check_pjds(a, b_r, 0, lay, 0);
                    check_pjds(a, b_r, 0, lay, -1);
                    check_pjds(a, b_r, 0, lay, 64);
                }
            for (int64_t w : {128, 256, 1024})
                for (int32_t split : {0, -1, 128}) check_pjds(a, 64, w, PJDS_LAYOUT_BLOCK, split);
            for (uint32_t k : {1u, 2u, 3u}) check_pjds(a, 64 >> k, 256, PJDS_LAYOUT_BLOCK | PJDS_LANES(k), 0);
            if (sh[0] == sh[1]) check_pjds(a, 64, 256, PJDS_LAYOUT_BLOCK | PJDS_SYMMETRIC, 0);
            check_split_and_ellr(a, r);
        }
    }
    check_refusals(r);
    std::printf("host driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
