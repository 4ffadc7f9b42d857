// The product inside an iterative solver that never leaves the permuted basis: m steps of
// the symmetric Lanczos recurrence run entirely on the GPU.
//
// The paper motivates pJDS by Krylov solvers that permute once before the iteration and
// once after it (Sect. 2.1).  With a matrix converted with PJDS_SYMMETRIC the product maps
// permuted vectors to permuted vectors, so the whole recurrence stays in that basis.  The
// Lanczos vectors are kept unnormalised, v_j = u_j / s_j (s_0 = |v|, s_j = beta_j), so no
// pass rescales a vector:
//
//     w = (1/s_j) A u_j - (beta_j / s_{j-1}) u_{j-1}   one pJDS product, both factors applied
//                                                     in its epilogue
//     alpha_j = (w . u_j) / s_j                       deterministic two-stage reduction; with
//                                                     x staged in LDS the product's workgroups
//                                                     sum w_i u_j[i] over their own rows (u_j[i]
//                                                     is staged), and every workgroup of the
//                                                     update adds those partial sums itself
//     w = w - (alpha_j / s_j) u_j;  t = w . w         one pass (the update)
//     beta_{j+1} = sqrt(t);  u_{j+1} = w              with x staged: added up by every
//                                                     workgroup of the next product, before
//                                                     its epilogue needs 1 / s_{j+1}
//
// Every scalar stays in device memory or is recomputed where it is needed, so a step needs no
// host synchronisation and a sequence of steps can be captured in a graph.  Reductions use a
// fixed grid and fixed summation trees, and a workgroup that adds another kernel's partial sums
// adds them in the same order as every other: results are reproducible bit for bit, with no
// device-scope fence or atomic.  With x staged in LDS a step is two kernels, the product and the
// update; vector passes per step besides the product's own x and y traffic: four (z read; w and
// u_j read and w written by the update), six with x through the caches (w and u_j read once
// more for alpha, in a kernel of its own, and two small kernels finish the scalars).
#include <algorithm>
#include <cmath>

#include "launch.h"

namespace pjds {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;     // fixed, so the summation order never depends on the device

__device__ __forceinline__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = kRedThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    return red[0];
}

// partial[b] = sum over this block's fixed share of a[i] * b[i]
__global__ __launch_bounds__(kRedThreads) void dot_partial_kernel(int64_t n, const double *__restrict__ a,
                                                                  const double *__restrict__ b,
                                                                  double *__restrict__ partial) {
    __shared__ double red[kRedThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(kRedThreads) + threadIdx.x; i < n; i += int64_t(kRedBlocks) * kRedThreads)
        s = __builtin_fma(a[i], b[i], s);
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// The update pass: alpha_j = (sum of the n_dot partials dot_part[] in a fixed order) * inv_s[0],
// added up by every workgroup (the same bits everywhere; workgroup 0 stores it in alpha_out[0]);
// then w = w - alpha_j inv_s[0] v and partial[b] = this workgroup's share of w . w (new w), each
// thread taking kUpdInFlight elements per round with all loads issued first.  The first
// round's loads go out before the partials are added, so their latency overlaps that sum.
constexpr int kUpdThreads = 1024;
constexpr int kUpdBlocks = 512;     // fixed, so the summation order never depends on the device
constexpr int kUpdInFlight = 4;
// Sum over the workgroup in a fixed order: xor butterfly inside each wave, then the waves in
// order (every thread returns the total).
__device__ __forceinline__ double block_sum_upd(double v, double *wsum) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();                                        // wsum free
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kUpdThreads / kWave; ++w) t += wsum[w];
    return t;
}
// VW = 2: elements in aligned pairs, 16-byte loads and stores (n even, every vector 16-byte
// aligned); a thread adds its elements' squares in element order either way.
template <int VW>
__global__ __launch_bounds__(kUpdThreads) void update_kernel(int64_t n, double *__restrict__ w,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ dot_part, int64_t n_dot,
                                                             const double *__restrict__ inv_s,
                                                             double *__restrict__ alpha_out,
                                                             double *__restrict__ partial) {
    typedef double Vd __attribute__((ext_vector_type(VW)));
    __shared__ double wsum[kUpdThreads / kWave];
    const int64_t nv = n / VW;                              // VW divides n
    const int64_t stride = int64_t(kUpdBlocks) * kUpdThreads;
    Vd *wp = reinterpret_cast<Vd *>(w);
    const Vd *vp = reinterpret_cast<const Vd *>(v);
    int64_t i0 = blockIdx.x * int64_t(kUpdThreads) + threadIdx.x;
    Vd wv[kUpdInFlight], vv[kUpdInFlight];
    auto load = [&](int64_t b) {
#pragma unroll
        for (int u = 0; u < kUpdInFlight; ++u) {
            const int64_t i = b + u * stride;
            wv[u] = i < nv ? wp[i] : Vd{};
            vv[u] = i < nv ? vp[i] : Vd{};
        }
    };
    load(i0);
    double d = 0.0;
    for (int64_t q = threadIdx.x; q < n_dot; q += kUpdThreads) d += dot_part[q];
    const double alpha = block_sum_upd(d, wsum) * inv_s[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha_out[0] = alpha;
    const double a = alpha * inv_s[0];
    double s = 0.0;
    for (;;) {
#pragma unroll
        for (int u = 0; u < kUpdInFlight; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < nv) {
                Vd r;
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    const double wi = __builtin_fma(-a, vv[u][e], wv[u][e]);
                    r[e] = wi;
                    s = __builtin_fma(wi, wi, s);
                }
                wp[i] = r;
            }
        }
        i0 += stride * kUpdInFlight;
        if (i0 >= nv) break;
        load(i0);
    }
    const double t = block_sum_upd(s, wsum);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Sum of n_part partials (fixed tree), then one of
//   kAlpha:  out[0] = sum * inv_s[0]                           (alpha_j = (w . u_j) / s_j)
//   kBeta:   b = sqrt(sum); out[0] = b; inv_next[0] = 1 / b;   (beta_{j+1}, 1 / s_{j+1},
//            zc_next[0] = b * inv_s[0]                          beta_{j+1} / s_j)
//   kNorm:   inv_next[0] = 1 / sqrt(sum)                       (1 / s_0)
enum FinishMode { kAlpha = 0, kBeta = 1, kNorm = 2 };
__global__ __launch_bounds__(kRedThreads) void finish_kernel(const double *__restrict__ partial, int64_t n_part,
                                                             int mode, const double *inv_s, double *out,
                                                             double *inv_next, double *zc_next) {
    __shared__ double red[kRedThreads];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n_part; q += kRedThreads) s += partial[q];
    const double t = block_sum(s, red);
    if (threadIdx.x != 0) return;
    if (mode == kAlpha) {
        out[0] = t * inv_s[0];
    } else if (mode == kBeta) {
        const double b = sqrt(t);
        out[0] = b;
        if (inv_next) inv_next[0] = 1.0 / b;
        if (zc_next) zc_next[0] = b * inv_s[0];
    } else {
        inv_next[0] = 1.0 / sqrt(t);
    }
}

// Partial sums a step leaves: w . u_j (the reduction grid's, or one per row tile of the staged
// product, tiles of at least 256 rows), then w . w (the update's) in a region of its own.
int64_t dot_slots(const pjds_info &in) { return std::max<int64_t>(kRedBlocks, ceil_div(in.n_pad, 256)); }
int64_t partial_slots(const pjds_info &in) { return dot_slots(in) + std::max(kRedBlocks, kUpdBlocks); }

__global__ void fill_kernel(int64_t n, double *p, double v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

}  // namespace
}  // namespace pjds

using namespace pjds;

extern "C" {

int pjds_lanczos_workspace(const pjds_info *info, int64_t *vector_bytes, int64_t *scratch_bytes) {
    if (!info || !vector_bytes || !scratch_bytes) return fail(PJDS_ERR_ARG, "NULL argument");
    *vector_bytes = 3 * std::max<int64_t>(info->n_rows, 1) * int64_t(sizeof(double));
    *scratch_bytes = (partial_slots(*info) + 8) * int64_t(sizeof(double));
    return PJDS_OK;
}

int pjds_lanczos(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                 const int32_t *d_col_p, const void *d_val_p, const int32_t *d_sched, void *d_work,
                 const double *d_v0, int32_t steps, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                 double *d_alpha, double *d_beta, void *d_vectors, void *d_scratch, void *stream) {
    if (int rc = check_product_info(info, PJDS_F64)) return rc;
    const pjds_info &in = *info;
    if (!(in.flags & PJDS_SYMMETRIC) || in.n_rows != in.n_cols)
        return fail(PJDS_ERR_ARG, "Lanczos needs a square matrix converted with PJDS_SYMMETRIC");
    if (steps < 0) return fail(PJDS_ERR_ARG, "steps %d", steps);
    if (flags & ~PJDS_ROW_LEN8) return fail(PJDS_ERR_ARG, "unknown Lanczos flags 0x%x", flags);
    if ((flags & PJDS_ROW_LEN8) && x_halo < 0)
        return fail(PJDS_ERR_ARG, "PJDS_ROW_LEN8 needs the staged product (x_halo >= 0)");
    if ((flags & PJDS_ROW_LEN8) && in.max_row_len > 255)
        return fail(PJDS_ERR_UNSUPPORTED, "PJDS_ROW_LEN8 with rows of %d entries (at most 255)", in.max_row_len);
    if (x_halo >= 0) {
        if (int rc = check_xlds(in, PJDS_F64, x_halo, tile_rows)) return rc;
    } else if (in.n_chunks && (!d_sched || !d_work)) {
        return fail(PJDS_ERR_ARG, "long rows need d_sched and d_work");
    }
    const int64_t n = in.n_rows;
    if (n == 0 || steps == 0) return PJDS_OK;
    if (!d_row_len || !d_offsets || !d_v0 || !d_alpha || !d_beta || !d_vectors || !d_scratch)
        return fail(PJDS_ERR_ARG, "NULL device array");
    if (in.nnz_stored && (!d_col_p || !d_val_p)) return fail(PJDS_ERR_ARG, "NULL device array");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *V = static_cast<double *>(d_vectors);
    double *part = static_cast<double *>(d_scratch);
    double *part_dot = part;                        // w . u_j partials
    double *part_nrm = part + dot_slots(in);        // w . w partials (and v . v before step 0)
    // device scalars, two slots each (step j reads slot j % 2 and writes the other)
    double *inv_s = part + partial_slots(in);       // 1 / s_j
    double *zc = inv_s + 2;                         // beta_j / s_{j-1} (x through the caches)
    const bool staged = x_halo >= 0;
    // the update in aligned pairs when every vector it touches is 16-byte aligned
    const bool pairs = n % 2 == 0 && (reinterpret_cast<uintptr_t>(d_v0) | reinterpret_cast<uintptr_t>(V)) % 16 == 0;
    // |v|^2 as partial sums (the staged product's first step adds them itself); beta_0 = 0
    hipLaunchKernelGGL(dot_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, d_v0, d_v0, part_nrm);
    if (!staged)
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kRedThreads), 0, s, part_nrm, int64_t(kRedBlocks), int(kNorm),
                           nullptr, nullptr, inv_s, nullptr);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, int64_t(1), d_beta, 0.0);
    for (int32_t j = 0; j < steps; ++j) {
        // u_0 is the caller's v (read only); then w of step j lands in V[(j + 1) % 3], which
        // held u_{j-2}
        const double *uj = j == 0 ? d_v0 : V + int64_t(j % 3) * n;
        const double *uprev = j == 0 ? nullptr : j == 1 ? d_v0 : V + int64_t((j - 1) % 3) * n;
        double *w = V + int64_t((j + 1) % 3) * n;
        double *inv_j = inv_s + (j & 1), *inv_n = inv_s + ((j + 1) & 1);
        // w = (1/s_j) A u_j - (beta_j / s_{j-1}) u_{j-1}
        EpiArgs ea;
        ea.z = uprev;
        int64_t n_dot = kRedBlocks;
        if (staged) {
            // 1 / s_j and beta_j / s_{j-1} from the partials of |u_j|^2 in every workgroup;
            // w . u_j as per-tile partial sums in the epilogue
            ea.norm_part = part_nrm;
            ea.n_norm = j == 0 ? kRedBlocks : kUpdBlocks;
            ea.inv_prev = j == 0 ? nullptr : inv_n;     // slot (j - 1) % 2 = (j + 1) % 2
            ea.inv_out = inv_j;
            ea.beta_out = j == 0 ? nullptr : d_beta + j;
            ea.dot_partial = part_dot;
            n_dot = xlds_tiles(in, tile_rows);
            launch_xlds(in, d_row_len, d_offsets, d_col_p, d_val_p, nullptr, PJDS_F64, uj, w, x_halo, tile_rows, ea,
                        PJDS_Y_PERMUTED | PJDS_TWO_ROWS | (flags & PJDS_ROW_LEN8), s);
        } else {
            ea.alpha_dev = inv_j;
            ea.beta_dev = zc + (j & 1);
            ea.bscale = -1.0;
            launch_spmv_epi(in, d_row_len, d_offsets, d_col_p, d_val_p, d_sched, d_work, PJDS_F64, uj, w, ea,
                            PJDS_Y_PERMUTED, s);
            hipLaunchKernelGGL(dot_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, w, uj, part_dot);
        }
        // alpha_j, then w -= (alpha_j / s_j) u_j with the partials of |w|^2
        if (pairs)
            hipLaunchKernelGGL(update_kernel<2>, dim3(kUpdBlocks), dim3(kUpdThreads), 0, s, n, w, uj, part_dot, n_dot,
                               inv_j, d_alpha + j, part_nrm);
        else
            hipLaunchKernelGGL(update_kernel<1>, dim3(kUpdBlocks), dim3(kUpdThreads), 0, s, n, w, uj, part_dot, n_dot,
                               inv_j, d_alpha + j, part_nrm);
        // beta_{j+1}: the next staged product adds the partials itself; otherwise, and after
        // the last step, one small kernel
        if (!staged || j == steps - 1)
            hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kRedThreads), 0, s, part_nrm, int64_t(kUpdBlocks),
                               int(kBeta), inv_j, d_beta + j + 1, staged ? nullptr : inv_n,
                               staged ? nullptr : zc + ((j + 1) & 1));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PJDS_ERR_HIP, "pjds_lanczos: %s", hipGetErrorString(e));
    return PJDS_OK;
}

}  // extern "C"
