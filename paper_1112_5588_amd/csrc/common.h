// Internal helpers shared by the host code and the kernel launchers of libpjds.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/pjds.h"

namespace pjds {

// Thread-local message of the last failing call (pjds_last_error).
void set_error(const char *fmt, ...);
const char *get_error();

// Record a message and return the status code, for `return fail(PJDS_ERR_ARG, "...")`.
int fail(int code, const char *fmt, ...);

// Number of host worker threads for conversion: PJDS_NUM_THREADS, else the hardware count
// (at most 32).
int host_threads();

// Run body(t, begin, end) over [0, n) split into contiguous ranges, one per thread.
template <class F>
void parallel_ranges(int64_t n, F body);

constexpr int kWave = 64;  // MI355X wavefront width

// Type-erased form of a product's epilogue y = alpha (A x) + b z (see spmv.hip).
struct EpiArgs {
    double alpha = 1.0, beta = 0.0;
    const void *z = nullptr;
    const void *beta_dev = nullptr;   // if set, b = bscale * (*beta_dev) read on the device
    double bscale = 0.0;
    const void *alpha_dev = nullptr;  // if set, the factor of A x is *alpha_dev, read on the device
    // if set (x staged in LDS, two rows per lane, a square matrix in the permuted basis, y
    // permuted): workgroup t of the product writes sum over its rows i of y_i * x_i to
    // dot_partial[t], in a fixed order (binary64)
    double *dot_partial = nullptr;
    // if set (the same staged two-rows product, as a Lanczos step): every workgroup adds the
    // n_norm values norm_part[] in a fixed order into t, and the epilogue uses alpha = 1 / b and
    // beta = -b * inv_prev[0] (beta only when z is set) with b = sqrt(t); the workgroup of the
    // first tile writes inv_out[0] = 1 / b and, if beta_out is set, beta_out[0] = b
    const double *norm_part = nullptr;
    int32_t n_norm = 0;
    const double *inv_prev = nullptr;
    double *inv_out = nullptr;
    double *beta_out = nullptr;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pjds

#include <thread>
#include <vector>

template <class F>
void pjds::parallel_ranges(int64_t n, F body) {
    int nt = host_threads();
    if (n < 65536 || nt <= 1) {
        body(0, int64_t(0), n);
        return;
    }
    if (nt > n) nt = int(n);
    std::vector<std::thread> pool;
    int64_t step = ceil_div(n, nt);
    for (int t = 0; t < nt; ++t) {
        int64_t b = t * step, e = b + step < n ? b + step : n;
        if (b >= e) break;
        pool.emplace_back([=] { body(t, b, e); });
    }
    for (auto &th : pool) th.join();
}
