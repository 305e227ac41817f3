// Coarse problem of the two-grid cycle (Eq. coarse, A_c = R_0 A R_0^T) with
// the Nicolaides coarse space: one vector per subdomain and PCE mode, the
// indicator of the nodes the subdomain owns.  Then
//     A_c = sum_i (Z^T K_i Z) (x) G_i =: sum_i C_i (x) G_i,
// the same Kronecker-sum structure as the fine operator on the graph of
// subdomains.  C_i is summed on the device from the fine values in a fixed
// order.  Two coarse solvers:
//   * mean-based exact: (C_0 (x) G_0)^{-1}, a dense n_sub x n_sub inverse;
//   * one V(1,1) cycle of smoothed-aggregation AMG on A_c (the paper's
//     2GV3 coarse solve uses BoomerAMG; its parameters are not given, so the
//     fixed definition below is used).  The hierarchy is built on the host
//     in FP64 (block-sparse matrices with dense P x P blocks, a few hundred
//     block-nodes); the cycle runs on the device.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>
#include <type_traits>

namespace sg {
namespace amgc {
constexpr double kTheta = 0.08;
constexpr double kOmegaS = 2.0 / 3.0;
constexpr int kMaxLevels = 4;
constexpr int kMinNodes = 8;
constexpr int kPowerIts = 15;
}  // namespace amgc
constexpr int kMaxInnerIts = 200;

// Host block-sparse matrix with dense P x P row-major blocks.
struct Bsr {
    int nr = 0, nc = 0, P = 0;
    std::vector<int32_t> ptr, col;
    std::vector<double> val;
    double* blk(size_t q) { return val.data() + q * (size_t)P * P; }
    const double* blk(size_t q) const { return val.data() + q * (size_t)P * P; }
};

struct AmgLevel {
    int nn = 0;
    // ap: A P (block rows of the level, columns of the next), for the
    // post-smoothing residual r - (A P) x_c
    DevBuf<int32_t> ap_ptr, ap_col;
    DevBuf<double> ap_val;
    DevBuf<int32_t> a_ptr, a_col, p_ptr, p_col, r_ptr, r_col;
    DevBuf<double> a_val, p_val, r_val, dinv64, x, b, r;
    DevBuf<double> xs;   // post-smoothed x of a level below the first
    DevBuf<float> dinv32;
    DevBuf<uint16_t> dinv16;
};

}  // namespace sg

struct sg_amg {
    int device = 0;
    sg_coarse_kind kind = SG_COARSE_AMG;
    sg_prec prec = SG_FP64;
    int n = 0, n_sub = 0, P = 0, L = 0;
    sg::DevBuf<int32_t> own_ptr, own_nodes, owner;
    int nslices = 0;
    sg::DevBuf<int32_t> slice_sub, slice_beg, slice_end, sub_slice_ptr;
    sg::DevBuf<double> slice_part;
    sg::DevBuf<double> afact;
    sg::DevBuf<double> c0inv;                 // mean-exact
    std::vector<sg::AmgLevel> lev;            // AMG levels (last = coarsest)
    sg::DevBuf<double> coarsest_inv;
    int coarsest_n = 0;
    std::vector<int32_t> h_nodes, h_agg0;
    std::vector<double> h_omegas;
    // inner Krylov coarse solve (amg_set_inner): basis V [(m+1) ld], flexible
    // directions Z [m ld], w [ld], and Hessenberg / rotations / scalars
    sg_inner_kind inner = SG_INNER_NONE;
    double inner_rtol = 0.0;
    int inner_max = 0;
    int64_t inner_ld = 0;
    sg::DevBuf<double> iV, iZ, iw, ismall;
    double* ipin = nullptr;                   // pinned host slot for one estimate
    mutable int64_t inner_calls = 0, inner_its = 0;
    mutable int inner_last = 0;
    // geometric coarse space (SG_COARSE_GEOMETRIC): P_0 by fine rows (three
    // (coarse node, weight) slots per fine node, weight 0 in unused slots),
    // P_0^T by coarse rows, and the coarse problem's own operator, RAS,
    // coarse correction and FGMRES workspace
    int ratio = 0, g_restart = 0, g_max = 0, g_graph = 1;
    double g_omega = 1.0;
    sg::DevBuf<int32_t> gp_col, gr_ptr, gr_col;
    sg::DevBuf<double> gp_val, gr_val;
    sg_op* gop = nullptr;
    sg_ras* gras = nullptr;
    sg_amg* gamg = nullptr;
    sg::DevBuf<char> gws;
    // (A Z) of the Nicolaides space for the operator it was built from
    // (values fixed): rows with a non-zero, their entries (subdomain, L_in
    // values), the triple table by (k, i, j) with per-(k, i) ranges, and E =
    // e_c G_i [L_in][n_sub][P] of the current coarse correction
    const sg_op* az_op = nullptr;
    int az_rows_n = 0;
    // entries grouped by subdomain (az_sptr ranges, values az_sval) so that
    // one work-group per subdomain forms E_s in LDS and the products of its
    // entries (into az_W [entry][P]); per row, the entries' positions az_rpos
    sg::DevBuf<int32_t> az_rows, az_ptr, az_rpos, az_sptr, az_kptr, az_tj;
    sg::DevBuf<double> az_sval, az_tv, az_W;
    ~sg_amg() {
        if (ipin) (void)hipHostFree(ipin);
        if (gamg) sg_destroy_amg(gamg);
        if (gras) sg_destroy_ras(gras);
        if (gop) sg_destroy_op(gop);
    }
};

namespace sg {
namespace {

constexpr int kBlk = 128;   // threads per block-row kernel (P <= 128)

__global__ void coarse_entries_kernel(int64_t nce, int L, const int64_t* __restrict__ cptr,
                                      const int64_t* __restrict__ fine,
                                      const double* __restrict__ vals, double* __restrict__ C) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nce * L) return;
    int64_t ce = idx / L;
    int i = (int)(idx - ce * L);
    double acc = 0.0;
    for (int64_t q = cptr[ce]; q < cptr[ce + 1]; ++q) acc += vals[fine[q] * L + i];
    C[idx] = acc;
}

// r_c[s, k] = sum over owned nodes a of R[a, k]: stage 1 sums slices of
// kSlice owned nodes per work-group, stage 2 adds the slices of a subdomain
// in order (fixed summation order, no atomics).
constexpr int kSlice = 64;
__global__ __launch_bounds__(256) void restrict_partial_kernel(
    int P, int nslices, const int32_t* __restrict__ slice_sub, const int32_t* __restrict__ slice_beg,
    const int32_t* __restrict__ slice_end, const int32_t* __restrict__ own_nodes,
    const double* __restrict__ R, double* __restrict__ part) {
    __shared__ double red[256];
    const int sl = blockIdx.x, tid = threadIdx.x;
    const int stripes = 256 / P;
    const int k = tid % P, st = tid / P;
    double acc = 0.0;
    if (st < stripes) {
        // the nodes q = beg + st, beg + st + stripes, ... added in order; the
        // loads of four of them are issued before their additions
        const int end = slice_end[sl];
        for (int q = slice_beg[sl] + st; q < end; q += 4 * stripes) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int qq = q + u * stripes;
                v[u] = qq < end ? R[(size_t)own_nodes[qq] * P + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u * stripes < end) acc += v[u];
        }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < P) {
        double t = 0.0;
        for (int w = 0; w < stripes; ++w) t += red[w * P + tid];
        part[(size_t)sl * P + tid] = t;
    }
}

__global__ void restrict_final_kernel(int ns, int P, const int32_t* __restrict__ sub_slice_ptr,
                                      const double* __restrict__ part, double* __restrict__ rc) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ns * P) return;
    int s = idx / P, k = idx - (idx / P) * P;
    double t = 0.0;
    for (int q = sub_slice_ptr[s]; q < sub_slice_ptr[s + 1]; ++q) t += part[(size_t)q * P + k];
    rc[idx] = t;
}

// Y[a, k] += e_c[owner(a), k]; total = n P < 2^31 (checked by the caller),
// so the node index comes from a 32-bit division.
__global__ void prolong_add_kernel(int total, int P, const int32_t* __restrict__ owner,
                                   const double* __restrict__ ec, double* __restrict__ Y) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int a = (int)((unsigned)idx / (unsigned)P);
    const int k = idx - a * P;
    Y[idx] += ec[(size_t)owner[a] * P + k];
}

// Geometric coarse space.  r_c[I, k] = sum_q w_q R[a_q, k] over the fine
// nodes a_q of coarse row I of P_0^T (one work-group per coarse node, the
// entries q = beg + st, beg + st + stripes, ... per stripe, stripes added in
// order), and Y[a, k] += sum_{slots} w e_c[I, k] over the (at most three)
// coarse nodes interpolated at fine node a.
__global__ __launch_bounds__(256) void geo_restrict_kernel(
    int P, const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
    const double* __restrict__ rval, const double* __restrict__ R, double* __restrict__ rc) {
    __shared__ double red[256];
    const int I = blockIdx.x, tid = threadIdx.x;
    const int stripes = 256 / P;
    const int k = tid % P, st = tid / P;
    double acc = 0.0;
    if (st < stripes) {
        const int end = rptr[I + 1];
        for (int q = rptr[I] + st; q < end; q += stripes)
            acc = fma(rval[q], R[(size_t)rcol[q] * P + k], acc);
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < P) {
        double t = 0.0;
        for (int w = 0; w < stripes; ++w) t += red[w * P + tid];
        rc[(size_t)I * P + tid] = t;
    }
}

__global__ void geo_prolong_add_kernel(int total, int P, const int32_t* __restrict__ pcol,
                                       const double* __restrict__ pval,
                                       const double* __restrict__ ec, double* __restrict__ Y) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int a = (int)((unsigned)idx / (unsigned)P);
    const int k = idx - a * P;
    double t = Y[idx];
#pragma unroll
    for (int q = 0; q < 3; ++q) t = fma(pval[3 * a + q], ec[(size_t)pcol[3 * a + q] * P + k], t);
    Y[idx] = t;
}

// One work-group per subdomain s: E_s[i][k] = sum_j m_ijk e_c[s, j] in LDS
// (one thread per (i, k) over the triples of (k, i), kiptr ranges of the
// table sorted by k, i, j), then W[q][k] = sum_i AZ_i(q) E_s[i][k] for the
// entries q of column s.
__global__ __launch_bounds__(1024) void az_entry_kernel(int P, int L,
                                                       const int32_t* __restrict__ sptr,
                                                       const double* __restrict__ sval,
                                                       const int32_t* __restrict__ kiptr,
                                                       const int32_t* __restrict__ tj,
                                                       const double* __restrict__ tv,
                                                       const double* __restrict__ ec,
                                                       double* __restrict__ W) {
    extern __shared__ double Es[];                 // [L][P]
    const int sd = blockIdx.x;
    const int q0 = sptr[sd], q1 = sptr[sd + 1];
    if (q0 == q1) return;
    for (int x = threadIdx.x; x < L * P; x += blockDim.x) {
        const int i = x / P, k = x - i * P;
        double acc = 0.0;
        for (int t = kiptr[k * L + i]; t < kiptr[k * L + i + 1]; ++t)
            acc = fma(tv[t], ec[(size_t)sd * P + tj[t]], acc);
        Es[x] = acc;
    }
    __syncthreads();
    // the loads of eight input terms are issued before their products
    for (int x = threadIdx.x; x < (q1 - q0) * P; x += blockDim.x) {
        const int qq = x / P, k = x - qq * P;
        const double* v = sval + (size_t)(q0 + qq) * L;
        double acc = 0.0;
        for (int i0 = 0; i0 < L; i0 += 8) {
            double vv[8], ee[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = i0 + u < L;
                vv[u] = in ? v[i0 + u] : 0.0;
                ee[u] = in ? Es[(i0 + u) * P + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fma(vv[u], ee[u], acc);
        }
        W[(size_t)(q0 + qq) * P + k] = acc;
    }
}

// T[a, k] -= sum of W[q][k] over the row's entries q (column order), one
// thread per (row, k).
__global__ void az_rows_kernel(int nrows, int P, const int32_t* __restrict__ rows,
                               const int32_t* __restrict__ ptr, const int32_t* __restrict__ rpos,
                               const double* __restrict__ W, double* __restrict__ T) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * P) return;
    const int r = idx / P, k = idx - r * P;
    double acc = 0.0;
    for (int e = ptr[r]; e < ptr[r + 1]; ++e) acc += W[(size_t)rpos[e] * P + k];
    T[(size_t)rows[r] * P + k] -= acc;
}

// x[s, k] = sum_t C0inv[s, t] b[t, k] / alpha_k!
__global__ void mean_exact_kernel(int ns, int P, const double* __restrict__ inv,
                                  const double* __restrict__ afact, const double* __restrict__ b,
                                  double* __restrict__ x) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ns * P) return;
    int s = idx / P, k = idx - (idx / P) * P;
    double acc = 0.0;
    for (int t = 0; t < ns; ++t) acc += inv[(size_t)s * ns + t] * b[(size_t)t * P + k];
    x[idx] = acc / afact[k];
}

// y = beta * c + alpha * A x   (block-sparse, dense P x P blocks).  One
// work-group of kBlkMv threads per block-row: thread (k, part) sums, for
// output row k, the (block, column) pairs part, part + nparts, ... of the
// block row (a few independent loads per thread), then the parts are added
// in a fixed order through LDS.  Blocks stored by rows (kColMajor false) or
// by columns (the restriction, whose block rows hold many blocks).
constexpr int kBlkMv = 1024;

__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// D_s^{-1} r_s (block-Jacobi) spread over a work-group of nthreads:
// thread (k, pi) sums columns pi, pi + np, ... of row k (np = nthreads / P),
// then the np partial sums of a row are added in order.  rs and part are in
// LDS (part: nthreads entries); every thread of the group calls it.  FP32
// accumulation for FP32 and BF16 blocks.
template <class TS>
__device__ inline double jacobi_par(int P, const TS* __restrict__ blk, const double* rs,
                                    double* part, int nthreads) {
    const int tid = threadIdx.x, np = nthreads / P;
    const int k = tid % P, pi = tid / P;
    double a = 0.0;
    if (pi < np) {
        if constexpr (sizeof(TS) == 8) {
            for (int j = pi; j < P; j += np) a = fma((double)blk[(size_t)k * P + j], rs[j], a);
        } else {
            float f = 0.0f;
            for (int j = pi; j < P; j += np) {
                float d;
                if constexpr (sizeof(TS) == 4) d = (float)blk[(size_t)k * P + j];
                else d = bf16_to_f((uint16_t)blk[(size_t)k * P + j]);
                f = fmaf(d, (float)rs[j], f);
            }
            a = (double)f;
        }
    }
    part[tid] = a;
    __syncthreads();
    double t = 0.0;
    if (tid < P)
        for (int w = 0; w < np; ++w) t += part[w * P + tid];
    __syncthreads();
    return t;
}

// TJ (not void): the work-group then also applies the block-Jacobi step
// xj_s = beta_j xo_s + omega_j Dinv_s y_s to the block row it produced (the
// smoother is block-diagonal, so no other row is needed): the pre-smoothing
// of the next level after a restriction (beta_j = 0), or the post-smoothing
// after a residual, whose input x the other work-groups still read: xj must
// then be another buffer than x (xo = x).
template <bool kColMajor, class TJ>
__global__ __launch_bounds__(kBlkMv) void bsr_mv_kernel(int P, const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ x, double* y,
                                                        double alpha, double beta, const double* c,
                                                        const TJ* __restrict__ dinv, double* xj,
                                                        const double* xo, double omega_j,
                                                        double beta_j) {
    __shared__ double part[kBlkMv];
    __shared__ double ys[kBlk];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nparts = kBlkMv / P;
    const int k = tid % P, pi = tid / P;
    // thread (k, pi) takes the (block, column) pairs e = pi, pi + nparts, ...
    // of the row: independent loads, a few per thread, issued together
    double acc = 0.0;
    if (pi < nparts) {
        const int q0 = ptr[s], tot = (ptr[s + 1] - q0) * P;
#pragma unroll 4
        for (int e = pi; e < tot; e += nparts) {
            const int qq = e / P, j = e - qq * P;
            const int q = q0 + qq;
            const double a = val[(size_t)q * P * P + (kColMajor ? (size_t)j * P + k : (size_t)k * P + j)];
            acc = fma(a, x[(size_t)col[q] * P + j], acc);
        }
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < P) {
        double t = 0.0;
        for (int w = 0; w < nparts; ++w) t += part[w * P + tid];
        const size_t o = (size_t)s * P + tid;
        double v = alpha * t;
        if (beta != 0.0) v = fma(beta, c[o], v);
        y[o] = v;
        if constexpr (!std::is_void_v<TJ>) ys[tid] = v;
    }
    if constexpr (!std::is_void_v<TJ>) {
        __syncthreads();
        const double acc = jacobi_par<TJ>(P, dinv + (size_t)s * P * P, ys, part, kBlkMv);
        if (tid < P) {
            const size_t o = (size_t)s * P + tid;
            xj[o] = (beta_j != 0.0 ? beta_j * xo[o] : 0.0) + omega_j * acc;
        }
    }
}

// The coarse correction and post-smoothing of one level, per block row s:
// p = (P x_c)_s, q = ((A P) x_c)_s, r1 = r0_s - q (= b - A (x + P x_c)),
// out_s = x_s + p + omega D_s^{-1} r1; r0 is the residual of the iterate
// before the correction.  out may equal x (each row reads only its own x).
template <class TJ>
__global__ __launch_bounds__(kBlkMv) void bsr_post_kernel(
    int P, const int32_t* __restrict__ pptr, const int32_t* __restrict__ pcol,
    const double* __restrict__ pval, const int32_t* __restrict__ aptr,
    const int32_t* __restrict__ acol, const double* __restrict__ aval,
    const double* __restrict__ xc, const double* __restrict__ r0, const double* x, double* out,
    const TJ* __restrict__ dinv, double omega) {
    __shared__ double part[kBlkMv];
    __shared__ double ps[kBlk], rs[kBlk];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nparts = kBlkMv / P;
    const int k = tid % P, pi = tid / P;
    auto row_product = [&](const int32_t* ptr, const int32_t* col, const double* val) {
        double acc = 0.0;
        if (pi < nparts) {
            const int q0 = ptr[s], tot = (ptr[s + 1] - q0) * P;
#pragma unroll 4
            for (int e = pi; e < tot; e += nparts) {
                const int qq = e / P, j = e - qq * P;
                const int q = q0 + qq;
                acc = fma(val[(size_t)q * P * P + (size_t)k * P + j], xc[(size_t)col[q] * P + j], acc);
            }
        }
        part[tid] = acc;
        __syncthreads();
        double t = 0.0;
        if (tid < P)
            for (int w = 0; w < nparts; ++w) t += part[w * P + tid];
        __syncthreads();
        return t;
    };
    const double p = row_product(pptr, pcol, pval);
    const double q = row_product(aptr, acol, aval);
    if (tid < P) {
        ps[tid] = p;
        rs[tid] = r0[(size_t)s * P + tid] - q;
    }
    __syncthreads();
    const double acc = jacobi_par<TJ>(P, dinv + (size_t)s * P * P, rs, part, kBlkMv);
    if (tid < P) {
        const size_t o = (size_t)s * P + tid;
        out[o] = x[o] + ps[tid] + omega * acc;
    }
}

// x_s = beta * x_s + omega * D_s^{-1} r_s  (block-Jacobi), D^{-1} in TS.
template <class TS>
__global__ __launch_bounds__(kBlk) void jacobi_kernel(int P, const TS* __restrict__ dinv,
                                                      const double* __restrict__ r, double* x,
                                                      double omega, double beta) {
    __shared__ double rs[kBlk], part[kBlk];
    const int s = blockIdx.x, tid = threadIdx.x;
    if (tid < P) rs[tid] = r[(size_t)s * P + tid];
    __syncthreads();
    const double acc = jacobi_par<TS>(P, dinv + (size_t)s * P * P, rs, part, kBlk);
    if (tid < P) {
        const size_t o = (size_t)s * P + tid;
        x[o] = (beta != 0.0 ? beta * x[o] : 0.0) + omega * acc;
    }
}

// x = A b for the dense column-major coarsest inverse: a work-group of 256
// threads per 32 rows, thread (r, part) summing columns part, part + 8, ...;
// the 8 partial sums of a row are added in a fixed order.
constexpr int kDenseRows = 32, kDenseParts = 8;
__global__ __launch_bounds__(kDenseRows * kDenseParts) void dense_mv_kernel(
    int N, const double* __restrict__ A, const double* __restrict__ b, double* __restrict__ x) {
    __shared__ double part[kDenseParts][kDenseRows];
    const int r = threadIdx.x % kDenseRows, pt = threadIdx.x / kDenseRows;
    const int i = blockIdx.x * kDenseRows + r;
    double acc = 0.0;
    if (i < N)
        for (int j = pt; j < N; j += kDenseParts) acc = fma(A[(size_t)j * N + i], b[j], acc);
    part[pt][r] = acc;
    __syncthreads();
    if (pt == 0 && i < N) {
        double t = 0.0;
        for (int q = 0; q < kDenseParts; ++q) t += part[q][r];
        x[i] = t;
    }
}

uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- host FP64
// In-place inverse of a dense SPD-or-general N x N matrix (Gauss-Jordan with
// partial pivoting).  Throws SG_ERR_NUMERIC on a zero pivot.
void invert_dense(std::vector<double>& A, int N) {
    std::vector<int> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<double> I((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) I[(size_t)i * N + i] = 1.0;
    for (int k = 0; k < N; ++k) {
        int piv = k;
        for (int i = k + 1; i < N; ++i)
            if (std::fabs(A[(size_t)i * N + k]) > std::fabs(A[(size_t)piv * N + k])) piv = i;
        double pv = A[(size_t)piv * N + k];
        if (!(std::fabs(pv) > 0.0) || !std::isfinite(pv))
            SG_THROW(SG_ERR_NUMERIC, "singular block in the coarse hierarchy");
        if (piv != k)
            for (int j = 0; j < N; ++j) {
                std::swap(A[(size_t)k * N + j], A[(size_t)piv * N + j]);
                std::swap(I[(size_t)k * N + j], I[(size_t)piv * N + j]);
            }
        double ip = 1.0 / A[(size_t)k * N + k];
        for (int j = 0; j < N; ++j) {
            A[(size_t)k * N + j] *= ip;
            I[(size_t)k * N + j] *= ip;
        }
        for (int i = 0; i < N; ++i) {
            if (i == k) continue;
            double f = A[(size_t)i * N + k];
            if (f == 0.0) continue;
            for (int j = 0; j < N; ++j) {
                A[(size_t)i * N + j] -= f * A[(size_t)k * N + j];
                I[(size_t)i * N + j] -= f * I[(size_t)k * N + j];
            }
        }
    }
    A.swap(I);
}

// C (+)= A * B for dense P x P blocks
inline void gemm_acc(int P, const double* A, const double* B, double* C) {
    for (int i = 0; i < P; ++i)
        for (int k = 0; k < P; ++k) {
            double a = A[(size_t)i * P + k];
            if (a == 0.0) continue;
            const double* b = B + (size_t)k * P;
            double* c = C + (size_t)i * P;
            for (int j = 0; j < P; ++j) c[j] += a * b[j];
        }
}

Bsr bsr_mul(const Bsr& A, const Bsr& B) {
    const int P = A.P;
    Bsr C;
    C.nr = A.nr; C.nc = B.nc; C.P = P;
    C.ptr.assign(A.nr + 1, 0);
    std::vector<double> acc;
    for (int s = 0; s < A.nr; ++s) {
        std::map<int, size_t> slot;
        std::vector<double> blocks;
        for (int q = A.ptr[s]; q < A.ptr[s + 1]; ++q) {
            int t = A.col[q];
            for (int q2 = B.ptr[t]; q2 < B.ptr[t + 1]; ++q2) {
                int u = B.col[q2];
                auto it = slot.find(u);
                size_t idx;
                if (it == slot.end()) {
                    idx = slot.size();
                    slot[u] = idx;
                    blocks.resize((idx + 1) * (size_t)P * P, 0.0);
                } else {
                    idx = it->second;
                }
                gemm_acc(P, A.blk(q), B.blk(q2), blocks.data() + idx * (size_t)P * P);
            }
        }
        for (auto& kv : slot) {
            C.col.push_back(kv.first);
            C.val.insert(C.val.end(), blocks.begin() + kv.second * (size_t)P * P,
                         blocks.begin() + (kv.second + 1) * (size_t)P * P);
        }
        C.ptr[s + 1] = (int32_t)C.col.size();
    }
    return C;
}

Bsr bsr_transpose(const Bsr& A) {
    const int P = A.P;
    Bsr T;
    T.nr = A.nc; T.nc = A.nr; T.P = P;
    T.ptr.assign(A.nc + 1, 0);
    for (int q = 0; q < (int)A.col.size(); ++q) T.ptr[A.col[q] + 1]++;
    for (int i = 0; i < A.nc; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    std::vector<int32_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int s = 0; s < A.nr; ++s)
        for (int q = A.ptr[s]; q < A.ptr[s + 1]; ++q) {
            int d = fill[A.col[q]]++;
            T.col[d] = s;
            const double* src = A.blk(q);
            double* dst = T.blk(d);
            for (int i = 0; i < P; ++i)
                for (int j = 0; j < P; ++j) dst[(size_t)j * P + i] = src[(size_t)i * P + j];
        }
    return T;
}

void bsr_apply(const Bsr& A, const std::vector<double>& x, std::vector<double>& y) {
    const int P = A.P;
    y.assign((size_t)A.nr * P, 0.0);
    for (int s = 0; s < A.nr; ++s)
        for (int q = A.ptr[s]; q < A.ptr[s + 1]; ++q) {
            const double* b = A.blk(q);
            const double* xv = x.data() + (size_t)A.col[q] * P;
            for (int i = 0; i < P; ++i) {
                double acc = 0.0;
                for (int j = 0; j < P; ++j) acc += b[(size_t)i * P + j] * xv[j];
                y[(size_t)s * P + i] += acc;
            }
        }
}

std::vector<int> aggregate(const Bsr& A) {
    const int nn = A.nr;
    std::vector<double> diag(nn, 0.0);
    for (int s = 0; s < nn; ++s)
        for (int q = A.ptr[s]; q < A.ptr[s + 1]; ++q)
            if (A.col[q] == s) diag[s] = std::fabs(A.blk(q)[0]);
    std::vector<std::vector<std::pair<int, double>>> nb(nn);
    for (int s = 0; s < nn; ++s)
        for (int q = A.ptr[s]; q < A.ptr[s + 1]; ++q) {
            int t = A.col[q];
            double v = A.blk(q)[0];
            if (t != s && v != 0.0 && std::fabs(v) >= amgc::kTheta * std::sqrt(diag[s] * diag[t]))
                nb[s].push_back({t, std::fabs(v)});
        }
    std::vector<int> agg(nn, -1);
    int na = 0;
    for (int i = 0; i < nn; ++i) {      // pass 1
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (auto& p : nb[i]) free_nb &= agg[p.first] < 0;
        if (!free_nb) continue;
        agg[i] = na;
        for (auto& p : nb[i]) agg[p.first] = na;
        ++na;
    }
    std::vector<int> snap = agg;
    for (int i = 0; i < nn; ++i) {      // pass 2
        if (agg[i] >= 0) continue;
        int best = -1;
        double bv = -1.0;
        for (auto& p : nb[i])
            if (snap[p.first] >= 0 && p.second > bv) { best = p.first; bv = p.second; }
        if (best >= 0) agg[i] = snap[best];
    }
    for (int i = 0; i < nn; ++i) {      // pass 3
        if (agg[i] >= 0) continue;
        agg[i] = na;
        for (auto& p : nb[i])
            if (agg[p.first] < 0) agg[p.first] = na;
        ++na;
    }
    return agg;
}

// Column-major copy of dense P x P blocks (the coarsest inverse is read by
// columns, so that consecutive threads read consecutive words).
template <class T>
std::vector<T> transpose_blocks(const std::vector<T>& v, int P) {
    std::vector<T> t(v.size());
    const size_t bs = (size_t)P * P;
    for (size_t b0 = 0; b0 < v.size(); b0 += bs)
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j) t[b0 + (size_t)j * P + i] = v[b0 + (size_t)i * P + j];
    return t;
}

// col_major: store every P x P block by columns (the layout bsr_mv_kernel
// reads with kColMajor).
void upload_bsr(const Bsr& A, DevBuf<int32_t>& ptr, DevBuf<int32_t>& col, DevBuf<double>& val,
                hipStream_t s, bool col_major = false) {
    ptr.upload(A.ptr, s);
    col.upload(A.col, s);
    if (!col_major) {
        val.upload(A.val, s);
        return;
    }
    const size_t nb = A.col.size();
    const int P = A.P;
    std::vector<double> t(A.val.size());
    for (size_t q = 0; q < nb; ++q)
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j)
                t[q * P * P + (size_t)j * P + i] = A.val[q * P * P + (size_t)i * P + j];
    val.upload(t, s);
    HIP_OK(hipStreamSynchronize(s));   // t is freed on return
}

}  // namespace

// One V(1,1)-cycle from level l: pre-smoothing x = omega D^{-1} b (already done
// by the restriction that produced b when pre_done), residual, restriction,
// the coarser cycle, prolongation, residual and post-smoothing; returns the
// buffer that holds the result.  Below level 0 the smoothing steps run in
// the work-groups of the block product before them (bsr_mv_kernel with a
// Jacobi inverse; the post-smoothed x goes to the level's xs, since the
// residual's other work-groups still read x): 15 launches for four levels
// instead of 19, with the same arithmetic.
const double* amg_vcycle_level(const sg_amg* a, int l, const double* b, double* x, hipStream_t s,
                               bool pre_done) {
    const int P = a->P;
    const AmgLevel& L = a->lev[l];
    const int nl = (int)a->lev.size();
    if (l == nl - 1) {
        int N = a->coarsest_n;
        dense_mv_kernel<<<(N + kDenseRows - 1) / kDenseRows, kDenseRows * kDenseParts, 0, s>>>(
            N, a->coarsest_inv.p, b, x);
        HIP_LAUNCH_OK();
        return x;
    }
    const AmgLevel& C = a->lev[l + 1];
    const double w = amgc::kOmegaS;
    // block product y = beta c + alpha M xin on a pattern; with jl >= 0 also
    // xj = beta_j xo + w Dinv_jl y on the rows it produces
    auto mv = [&](bool col_major, int nrows, const DevBuf<int32_t>& ptr, const DevBuf<int32_t>& col,
                  const DevBuf<double>& val, const double* xin, double* y, double alpha,
                  double beta, const double* c, int jl, double* xj, const double* xo,
                  double beta_j) {
        if (jl < 0) {
            if (col_major)
                bsr_mv_kernel<true, void><<<nrows, kBlkMv, 0, s>>>(
                    P, ptr.p, col.p, val.p, xin, y, alpha, beta, c, nullptr, nullptr, nullptr,
                    0.0, 0.0);
            else
                bsr_mv_kernel<false, void><<<nrows, kBlkMv, 0, s>>>(
                    P, ptr.p, col.p, val.p, xin, y, alpha, beta, c, nullptr, nullptr, nullptr,
                    0.0, 0.0);
        } else {
            const AmgLevel& J = a->lev[jl];
#define SG_BSR_J(CM, TS, DINV)                                                                     \
    bsr_mv_kernel<CM, TS><<<nrows, kBlkMv, 0, s>>>(P, ptr.p, col.p, val.p, xin, y, alpha, beta, c, \
                                                   DINV, xj, xo, w, beta_j)
            if (a->prec == SG_FP64) {
                if (col_major) SG_BSR_J(true, double, J.dinv64.p);
                else SG_BSR_J(false, double, J.dinv64.p);
            } else if (a->prec == SG_FP32) {
                if (col_major) SG_BSR_J(true, float, J.dinv32.p);
                else SG_BSR_J(false, float, J.dinv32.p);
            } else {
                if (col_major) SG_BSR_J(true, uint16_t, J.dinv16.p);
                else SG_BSR_J(false, uint16_t, J.dinv16.p);
            }
#undef SG_BSR_J
        }
        HIP_LAUNCH_OK();
    };
    auto jacobi = [&](const double* r, double beta) {
        if (a->prec == SG_FP64)
            jacobi_kernel<double><<<L.nn, kBlk, 0, s>>>(P, L.dinv64.p, r, x, w, beta);
        else if (a->prec == SG_FP32)
            jacobi_kernel<float><<<L.nn, kBlk, 0, s>>>(P, L.dinv32.p, r, x, w, beta);
        else
            jacobi_kernel<uint16_t><<<L.nn, kBlk, 0, s>>>(P, L.dinv16.p, r, x, w, beta);
        HIP_LAUNCH_OK();
    };
    if (!pre_done) jacobi(b, 0.0);
    // r = b - A x; b_c = R r, and x_c = w D_c^{-1} b_c unless level l + 1 is
    // the coarsest (solved exactly)
    mv(false, L.nn, L.a_ptr, L.a_col, L.a_val, x, L.r.p, -1.0, 1.0, b, -1, nullptr, nullptr, 0.0);
    const bool c_smooth = l + 1 < nl - 1;
    mv(true, C.nn, L.r_ptr, L.r_col, L.r_val, L.r.p, C.b.p, 1.0, 0.0, nullptr,
       c_smooth ? l + 1 : -1, c_smooth ? C.x.p : nullptr, nullptr, 0.0);
    const double* xc = amg_vcycle_level(a, l + 1, C.b.p, C.x.p, s, c_smooth);
    // x + P x_c + w D^{-1} (r - (A P) x_c) in one pass (into xs below level
    // 0), r = b - A x being the residual formed before the restriction
    if (L.ap_val.p) {
        double* out = l == 0 ? x : L.xs.p;
#define SG_POST(TS, DINV)                                                                          \
    bsr_post_kernel<TS><<<L.nn, kBlkMv, 0, s>>>(P, L.p_ptr.p, L.p_col.p, L.p_val.p, L.ap_ptr.p,    \
                                                L.ap_col.p, L.ap_val.p, xc, L.r.p, x, out, DINV, w)
        if (a->prec == SG_FP64) SG_POST(double, L.dinv64.p);
        else if (a->prec == SG_FP32) SG_POST(float, L.dinv32.p);
        else SG_POST(uint16_t, L.dinv16.p);
#undef SG_POST
        HIP_LAUNCH_OK();
        return out;
    }
    // x += P x_c; r = b - A x; then x + w D^{-1} r (into xs below level 0)
    mv(false, L.nn, L.p_ptr, L.p_col, L.p_val, xc, x, 1.0, 1.0, x, -1, nullptr, nullptr, 0.0);
    if (l == 0) {
        mv(false, L.nn, L.a_ptr, L.a_col, L.a_val, x, L.r.p, -1.0, 1.0, b, -1, nullptr, nullptr,
           0.0);
        jacobi(L.r.p, 1.0);
        return x;
    }
    mv(false, L.nn, L.a_ptr, L.a_col, L.a_val, x, L.r.p, -1.0, 1.0, b, l, L.xs.p, x, 1.0);
    return L.xs.p;
}

// ------------------------------------------------------------------ inner GMRES
// The coarse problem solved by GMRES on A_c (Sec. 3, the variants with an
// inner Krylov solve): right-preconditioned by one V-cycle (2GV3) or by the
// block Jacobi of the level-0 blocks, i.e. a non-overlapping one-level
// Schwarz method with one coarse node per subdomain (2GV2), flexible form
// (the directions z_j are kept), classical Gram-Schmidt with a second pass,
// Givens rotations.  The host reads the residual estimate after every step
// to stop at rtol ||b_c|| or after max_its steps (no restart).
constexpr int kIT = 256;

// c[i] = <V_i, w>, one work-group per basis vector (ldv = 0 and one
// work-group give <w, w> with V = w).
__global__ __launch_bounds__(kIT) void inner_dots_kernel(int N, int64_t ldv,
                                                         const double* __restrict__ V,
                                                         const double* __restrict__ w,
                                                         double* __restrict__ c) {
    __shared__ double sh[kIT / 64];
    const double* v = V + (int64_t)blockIdx.x * ldv;
    double a = 0.0;
    for (int t = threadIdx.x; t < N; t += kIT) a = fma(v[t], w[t], a);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int q = 0; q < kIT / 64; ++q) r += sh[q];
        c[blockIdx.x] = r;
    }
}

// w -= sum_{i<k} c_i V_i
__global__ __launch_bounds__(kIT) void inner_update_kernel(int N, int k, int64_t ldv,
                                                           const double* __restrict__ V,
                                                           const double* __restrict__ c,
                                                           double* __restrict__ w) {
    const int t = blockIdx.x * kIT + threadIdx.x;
    if (t >= N) return;
    double v = w[t];
    for (int i = 0; i < k; ++i) v = fma(-c[i], V[(int64_t)i * ldv + t], v);
    w[t] = v;
}

// Column j of the Hessenberg matrix (the two Gram-Schmidt passes c0 + c1,
// and ||w|| below the diagonal), the earlier rotations applied to it, a new
// rotation, and the residual estimate |g_{j+1}|: sc[0] = estimate,
// sc[1] = 1/||w|| (0 at a breakdown).
__global__ void inner_givens_kernel(int j, int m, const double* __restrict__ c0,
                                    const double* __restrict__ c1, const double* __restrict__ ww,
                                    double* H, double* cs, double* sn, double* g, double* sc) {
    if (threadIdx.x != 0) return;
    double* h = H + (size_t)j * (m + 1);
    for (int i = 0; i <= j; ++i) h[i] = c0[i] + c1[i];
    const double hn = sqrt(fmax(*ww, 0.0));
    sc[1] = hn > 0.0 ? 1.0 / hn : 0.0;
    h[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    const double r = hypot(h[j], hn);
    const double c = r > 0.0 ? h[j] / r : 1.0, sj = r > 0.0 ? hn / r : 0.0;
    cs[j] = c;
    sn[j] = sj;
    h[j] = r;
    h[j + 1] = 0.0;
    g[j + 1] = -sj * g[j];
    g[j] = c * g[j];
    sc[0] = fabs(g[j + 1]);
}

// y = H_k^{-1} g (upper triangular k x k), then the caller forms x = Z y
__global__ void inner_backsolve_kernel(int k, int m, const double* __restrict__ H,
                                       const double* __restrict__ g, double* __restrict__ y) {
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double v = g[i];
        for (int l = i + 1; l < k; ++l) v -= H[(size_t)l * (m + 1) + i] * y[l];
        const double d = H[(size_t)i * (m + 1) + i];
        y[i] = d != 0.0 ? v / d : 0.0;
    }
}

// x = sum_{i<k} y_i Z_i
__global__ __launch_bounds__(kIT) void inner_combine_kernel(int N, int k, int64_t ldz,
                                                            const double* __restrict__ Z,
                                                            const double* __restrict__ y,
                                                            double* __restrict__ x) {
    const int t = blockIdx.x * kIT + threadIdx.x;
    if (t >= N) return;
    double v = 0.0;
    for (int i = 0; i < k; ++i) v = fma(y[i], Z[(int64_t)i * ldz + t], v);
    x[t] = v;
}

// v = a w, a = *ad when ad is not null, else ah
__global__ __launch_bounds__(kIT) void inner_scale_kernel(int N, const double* ad, double ah,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ v) {
    const int t = blockIdx.x * kIT + threadIdx.x;
    if (t >= N) return;
    v[t] = (ad ? *ad : ah) * w[t];
}

__global__ void inner_init_kernel(int m, double beta, double* g) {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = i == 0 ? beta : 0.0;
}

bool inner_active(const sg_amg* a) {
    return (a->inner != SG_INNER_NONE && a->kind == SG_COARSE_AMG && a->lev.size() > 1) ||
           a->kind == SG_COARSE_GEOMETRIC;
}

void coarse_gmres(const sg_amg* a, const double* b, double* x, hipStream_t s) {
    const int P = a->P, N = a->n_sub * P, m = a->inner_max;
    const int64_t ld = a->inner_ld;
    const AmgLevel& L0 = a->lev[0];
    SG_REQUIRE(L0.nn == a->n_sub && a->iV.n >= (size_t)(m + 1) * ld && ld >= N,
               "inner GMRES workspace does not match the hierarchy");
    double* V = a->iV.p;
    double* Zd = a->iZ.p;
    double* w = a->iw.p;
    double* H = a->ismall.p;
    double* cs = H + (size_t)(m + 1) * m;
    double* sn = cs + (m + 1);
    double* g = sn + (m + 1);
    double* y = g + (m + 1);
    double* c0 = y + (m + 1);
    double* c1 = c0 + (m + 1);
    double* sc = c1 + (m + 1);                // estimate, 1/||w||, <w, w>
    const unsigned gN = (unsigned)((N + kIT - 1) / kIT);
    auto read_scalar = [&](const double* d) {
        HIP_OK(hipMemcpyAsync(a->ipin, d, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        return a->ipin[0];
    };
    inner_dots_kernel<<<1, kIT, 0, s>>>(N, 0, b, b, sc + 2);
    HIP_LAUNCH_OK();
    const double beta = std::sqrt(read_scalar(sc + 2));
    if (!std::isfinite(beta)) SG_THROW(SG_ERR_NUMERIC, "coarse right-hand side is not finite");
    ++a->inner_calls;
    a->inner_last = 0;
    if (beta == 0.0) {
        inner_scale_kernel<<<gN, kIT, 0, s>>>(N, nullptr, 0.0, b, x);
        HIP_LAUNCH_OK();
        return;
    }
    inner_init_kernel<<<1, 64, 0, s>>>(m, beta, g);
    HIP_LAUNCH_OK();
    inner_scale_kernel<<<gN, kIT, 0, s>>>(N, nullptr, 1.0 / beta, b, V);
    HIP_LAUNCH_OK();
    const double target = a->inner_rtol * beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
        const double* vj = V + (int64_t)j * ld;
        double* zj = Zd + (int64_t)j * ld;
        if (a->inner == SG_INNER_GMRES_AMG) {
            amg_vcycle_level(a, 0, vj, zj, s, false);
        } else if (a->prec == SG_FP64) {
            jacobi_kernel<double><<<L0.nn, kBlk, 0, s>>>(P, L0.dinv64.p, vj, zj, 1.0, 0.0);
        } else if (a->prec == SG_FP32) {
            jacobi_kernel<float><<<L0.nn, kBlk, 0, s>>>(P, L0.dinv32.p, vj, zj, 1.0, 0.0);
        } else {
            jacobi_kernel<uint16_t><<<L0.nn, kBlk, 0, s>>>(P, L0.dinv16.p, vj, zj, 1.0, 0.0);
        }
        HIP_LAUNCH_OK();
        bsr_mv_kernel<false, void><<<L0.nn, kBlkMv, 0, s>>>(
            P, L0.a_ptr.p, L0.a_col.p, L0.a_val.p, zj, w, 1.0, 0.0, nullptr, nullptr, nullptr,
            nullptr, 0.0, 0.0);
        HIP_LAUNCH_OK();
        inner_dots_kernel<<<j + 1, kIT, 0, s>>>(N, ld, V, w, c0);
        HIP_LAUNCH_OK();
        inner_update_kernel<<<gN, kIT, 0, s>>>(N, j + 1, ld, V, c0, w);
        HIP_LAUNCH_OK();
        inner_dots_kernel<<<j + 1, kIT, 0, s>>>(N, ld, V, w, c1);
        HIP_LAUNCH_OK();
        inner_update_kernel<<<gN, kIT, 0, s>>>(N, j + 1, ld, V, c1, w);
        HIP_LAUNCH_OK();
        inner_dots_kernel<<<1, kIT, 0, s>>>(N, 0, w, w, sc + 2);
        HIP_LAUNCH_OK();
        inner_givens_kernel<<<1, 64, 0, s>>>(j, m, c0, c1, sc + 2, H, cs, sn, g, sc);
        HIP_LAUNCH_OK();
        inner_scale_kernel<<<gN, kIT, 0, s>>>(N, sc + 1, 0.0, w, V + (int64_t)(j + 1) * ld);
        HIP_LAUNCH_OK();
        k = j + 1;
        const double est = read_scalar(sc);
        if (!(est > target)) break;           // converged, breakdown (0) or not finite
    }
    inner_backsolve_kernel<<<1, 64, 0, s>>>(k, m, H, g, y);
    HIP_LAUNCH_OK();
    inner_combine_kernel<<<gN, kIT, 0, s>>>(N, k, ld, Zd, y, x);
    HIP_LAUNCH_OK();
    a->inner_last = k;
    a->inner_its += k;
}

// Geometric coarse solve: FGMRES on A_c = P_0^T A P_0 from x = 0, stopped at
// ||b - A_c x|| <= rtol ||b|| or after g_max steps, preconditioned by the
// coarse problem's own RAS and (if any) its coarse correction.
void geometric_solve(const sg_amg* a, const double* b, double* x, hipStream_t s) {
    HIP_OK(hipMemsetAsync(x, 0, (size_t)a->n_sub * a->P * sizeof(double), s));
    sg_krylov_opts o{};
    o.restart = a->g_restart;
    o.max_it = a->g_max;
    o.rtol = a->inner_rtol;
    o.omega = a->g_omega;
    o.use_graph = a->g_graph;
    o.ortho = SG_ORTHO_CGS_DGKS;
    sg_krylov_stats st{};
    LinOp A;
    A.kron = a->gop; A.n = a->n_sub; A.P = a->P;
    (void)fgmres_core(A, a->gop, a->device, a->gras, a->gamg, b, x, &o, &st, a->gws.p, a->gws.n,
                      s);
    ++a->inner_calls;
    a->inner_last = st.iterations;
    a->inner_its += st.iterations;
}

// The coarse solve of the kind alone: one V-cycle, the exact mean-based
// solve, or the geometric coarse problem's FGMRES.
void coarse_solve_base(const sg_amg* a, const double* b, double* x, hipStream_t s) {
    if (a->kind == SG_COARSE_GEOMETRIC) {
        geometric_solve(a, b, x, s);
    } else if (a->kind == SG_COARSE_MEAN_EXACT) {
        int tot = a->n_sub * a->P;
        mean_exact_kernel<<<(tot + 127) / 128, 128, 0, s>>>(a->n_sub, a->P, a->c0inv.p, a->afact.p,
                                                             b, x);
        HIP_LAUNCH_OK();
    } else {
        amg_vcycle_level(a, 0, b, x, s, false);
    }
}

void coarse_solve(const sg_amg* a, const double* b, double* x, hipStream_t s) {
    if (a->kind != SG_COARSE_GEOMETRIC && inner_active(a)) coarse_gmres(a, b, x, s);
    else coarse_solve_base(a, b, x, s);
}

bool coarse_has_az(const sg_amg* a, const sg_op* op) {
    return op && a->az_op == op && op->fixed_values;
}

const int32_t* coarse_owner_dev(const sg_amg* a) {
    return (a->kind == SG_COARSE_MEAN_EXACT || a->kind == SG_COARSE_AMG) ? a->owner.p : nullptr;
}

bool coarse_residual_update(const sg_amg* a, const sg_op* op, const double* ec, double* T,
                            hipStream_t s) {
    if (!coarse_has_az(a, op)) return false;
    const int ns = a->n_sub, P = a->P, L = a->L;
    if (a->az_rows_n > 0) {
        az_entry_kernel<<<ns, 1024, (size_t)L * P * sizeof(double), s>>>(
            P, L, a->az_sptr.p, a->az_sval.p, a->az_kptr.p, a->az_tj.p, a->az_tv.p, ec, a->az_W.p);
        HIP_LAUNCH_OK();
        const int64_t tot = (int64_t)a->az_rows_n * P;
        az_rows_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
            a->az_rows_n, P, a->az_rows.p, a->az_ptr.p, a->az_rpos.p, a->az_W.p, T);
        HIP_LAUNCH_OK();
    }
    return true;
}

int amg_nsub(const sg_amg* a) { return a->n_sub; }
int amg_device(const sg_amg* a) { return a->device; }

void coarse_restrict(const sg_amg* a, const double* R, double* rc, hipStream_t s) {
    if (a->kind == SG_COARSE_GEOMETRIC) {
        geo_restrict_kernel<<<a->n_sub, 256, 0, s>>>(a->P, a->gr_ptr.p, a->gr_col.p, a->gr_val.p,
                                                      R, rc);
        HIP_LAUNCH_OK();
        return;
    }
    restrict_partial_kernel<<<a->nslices, 256, 0, s>>>(a->P, a->nslices, a->slice_sub.p,
                                                        a->slice_beg.p, a->slice_end.p,
                                                        a->own_nodes.p, R, a->slice_part.p);
    HIP_LAUNCH_OK();
    int tot = a->n_sub * a->P;
    restrict_final_kernel<<<(tot + 255) / 256, 256, 0, s>>>(a->n_sub, a->P, a->sub_slice_ptr.p,
                                                             a->slice_part.p, rc);
    HIP_LAUNCH_OK();
}

void coarse_prolong_add(const sg_amg* a, const double* ec, double* Y, hipStream_t s) {
    const int64_t tot = (int64_t)a->n * a->P;
    SG_REQUIRE(tot < (int64_t)INT32_MAX, "n*P = %lld exceeds the 32-bit prolongation index",
               (long long)tot);
    if (a->kind == SG_COARSE_GEOMETRIC) {
        geo_prolong_add_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
            (int)tot, a->P, a->gp_col.p, a->gp_val.p, ec, Y);
        HIP_LAUNCH_OK();
        return;
    }
    prolong_add_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((int)tot, a->P, a->owner.p,
                                                                       ec, Y);
    HIP_LAUNCH_OK();
}

}  // namespace sg

namespace sg {

// Owned-node lists (for the restriction), owner map (for the prolongation)
// and the restriction slices of the Nicolaides space of `owner`.
void amg_common_setup(sg_amg* a, const std::vector<int32_t>& owner, hipStream_t s) {
    const int n = a->n, ns = a->n_sub, P = a->P;
    // owned-node lists and owner map
    std::vector<int32_t> own_ptr(ns + 1, 0), own_nodes(n);
    for (int q = 0; q < n; ++q) own_ptr[owner[q] + 1]++;
    for (int q = 0; q < ns; ++q) own_ptr[q + 1] += own_ptr[q];
    {
        std::vector<int32_t> fill(own_ptr.begin(), own_ptr.end() - 1);
        for (int q = 0; q < n; ++q) own_nodes[fill[owner[q]]++] = q;
    }
    a->own_ptr.upload(own_ptr, s);
    a->own_nodes.upload(own_nodes, s);
    {
        std::vector<int32_t> ssub, sbeg, send, sptr(1, 0);
        for (int q = 0; q < ns; ++q) {
            for (int b0 = own_ptr[q]; b0 < own_ptr[q + 1]; b0 += kSlice) {
                ssub.push_back(q);
                sbeg.push_back(b0);
                send.push_back(std::min(b0 + kSlice, own_ptr[q + 1]));
            }
            sptr.push_back((int32_t)ssub.size());
        }
        a->nslices = (int)ssub.size();
        a->slice_sub.upload(ssub, s);
        a->slice_beg.upload(sbeg, s);
        a->slice_end.upload(send, s);
        a->sub_slice_ptr.upload(sptr, s);
        a->slice_part.alloc((size_t)a->nslices * P);
    }
    a->owner.upload(owner, s);
}

// The smoothed-aggregation hierarchy of a level-0 block matrix A (host, FP64).
void amg_build_hierarchy(sg_amg* a, Bsr A, hipStream_t s) {
    const int P = a->P, ns = a->n_sub;
    const sg_prec prec = a->prec;
    std::vector<Bsr> As{A}, Ps, APs;
    std::vector<std::vector<double>> Dinvs;
    while ((int)As.size() < amgc::kMaxLevels && As.back().nr > amgc::kMinNodes) {
        const Bsr& Al = As.back();
        std::vector<int> agg = aggregate(Al);
        int na = *std::max_element(agg.begin(), agg.end()) + 1;
        if (na >= Al.nr) break;
        if (As.size() == 1) a->h_agg0.assign(agg.begin(), agg.end());
        // block-diagonal inverse
        std::vector<double> Dinv((size_t)Al.nr * P * P);
        for (int r = 0; r < Al.nr; ++r) {
            bool found = false;
            for (int q = Al.ptr[r]; q < Al.ptr[r + 1]; ++q)
                if (Al.col[q] == r) {
                    std::vector<double> D(Al.blk(q), Al.blk(q) + (size_t)P * P);
                    invert_dense(D, P);
                    std::copy(D.begin(), D.end(), Dinv.begin() + (size_t)r * P * P);
                    found = true;
                }
            if (!found) SG_THROW(SG_ERR_NUMERIC, "missing diagonal block");
        }
        // spectral radius of D^{-1} A by power iteration from ones
        std::vector<double> v((size_t)Al.nr * P, 1.0), w, dw((size_t)Al.nr * P);
        double nv = std::sqrt((double)v.size());
        for (auto& e : v) e /= nv;
        double rho = 0.0;
        for (int it = 0; it < amgc::kPowerIts; ++it) {
            bsr_apply(Al, v, w);
            for (int r = 0; r < Al.nr; ++r)
                for (int i = 0; i < P; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < P; ++j)
                        acc += Dinv[(size_t)r * P * P + (size_t)i * P + j] * w[(size_t)r * P + j];
                    dw[(size_t)r * P + i] = acc;
                }
            double nw = 0.0;
            for (double e : dw) nw += e * e;
            rho = std::sqrt(nw);
            for (size_t q = 0; q < v.size(); ++q) v[q] = dw[q] / rho;
        }
        const double omega = (4.0 / 3.0) / rho;
        a->h_omegas.push_back(omega);
        // tentative prolongator and its smoothing P = T - omega D^{-1} A T
        std::vector<int> sizes(na, 0);
        for (int r = 0; r < Al.nr; ++r) sizes[agg[r]]++;
        Bsr Tm;
        Tm.nr = Al.nr; Tm.nc = na; Tm.P = P;
        Tm.ptr.resize(Al.nr + 1);
        Tm.val.assign((size_t)Al.nr * P * P, 0.0);
        for (int r = 0; r < Al.nr; ++r) {
            Tm.ptr[r] = r;
            Tm.col.push_back(agg[r]);
            double sc = 1.0 / std::sqrt((double)sizes[agg[r]]);
            for (int i = 0; i < P; ++i) Tm.blk(r)[(size_t)i * P + i] = sc;
        }
        Tm.ptr[Al.nr] = Al.nr;
        Bsr AT = bsr_mul(Al, Tm);
        Bsr Pm = AT;
        for (int r = 0; r < Al.nr; ++r)
            for (int q = AT.ptr[r]; q < AT.ptr[r + 1]; ++q) {
                std::vector<double> prod((size_t)P * P, 0.0);
                gemm_acc(P, Dinv.data() + (size_t)r * P * P, AT.blk(q), prod.data());
                double* dst = Pm.blk(q);
                for (size_t e = 0; e < prod.size(); ++e) dst[e] = -omega * prod[e];
                if (AT.col[q] == agg[r]) {
                    double sc = 1.0 / std::sqrt((double)sizes[agg[r]]);
                    for (int i = 0; i < P; ++i) dst[(size_t)i * P + i] += sc;
                }
            }
        Bsr AP = bsr_mul(Al, Pm);
        Bsr Pt = bsr_transpose(Pm);
        Bsr Ac = bsr_mul(Pt, AP);
        Dinvs.push_back(std::move(Dinv));
        Ps.push_back(std::move(Pm));
        APs.push_back(std::move(AP));
        As.push_back(std::move(Ac));
    }
    if (a->h_agg0.empty()) a->h_agg0.assign(ns, -1);
    const int nl = (int)As.size();
    a->lev.resize(nl);
    for (int l = 0; l < nl; ++l) {
        AmgLevel& Lv = a->lev[l];
        Lv.nn = As[l].nr;
        a->h_nodes.push_back(As[l].nr);
        Lv.x.alloc((size_t)Lv.nn * P);
        Lv.b.alloc((size_t)Lv.nn * P);
        Lv.r.alloc((size_t)Lv.nn * P);
        Lv.xs.alloc((size_t)Lv.nn * P);
        if (l < nl - 1) {
            upload_bsr(As[l], Lv.a_ptr, Lv.a_col, Lv.a_val, s);
            upload_bsr(Ps[l], Lv.p_ptr, Lv.p_col, Lv.p_val, s);
            upload_bsr(APs[l], Lv.ap_ptr, Lv.ap_col, Lv.ap_val, s);
            upload_bsr(bsr_transpose(Ps[l]), Lv.r_ptr, Lv.r_col, Lv.r_val, s, true);
            if (prec == SG_FP64) {
                Lv.dinv64.upload(Dinvs[l], s);
            } else if (prec == SG_FP32) {
                std::vector<float> f(Dinvs[l].begin(), Dinvs[l].end());
                Lv.dinv32.upload(f, s);
            } else {
                std::vector<uint16_t> h(Dinvs[l].size());
                for (size_t q = 0; q < h.size(); ++q) h[q] = host_bf16((float)Dinvs[l][q]);
                Lv.dinv16.upload(h, s);
            }
        }
        HIP_OK(hipStreamSynchronize(s));
    }
    // coarsest: dense FP64 inverse
    {
        const Bsr& Ac = As.back();
        const int N = Ac.nr * P;
        std::vector<double> D((size_t)N * N, 0.0);
        for (int r = 0; r < Ac.nr; ++r)
            for (int q = Ac.ptr[r]; q < Ac.ptr[r + 1]; ++q)
                for (int i = 0; i < P; ++i)
                    for (int j = 0; j < P; ++j)
                        D[(size_t)(r * P + i) * N + Ac.col[q] * P + j] = Ac.blk(q)[(size_t)i * P + j];
        invert_dense(D, N);
        a->coarsest_inv.upload(transpose_blocks(D, N), s);   // column-major
        a->coarsest_n = N;
    }
    HIP_OK(hipStreamSynchronize(s));
}

}  // namespace sg

using namespace sg;

namespace sg {

// (A Z) for the Nicolaides space: AZ_i[a, s] = sum of K_i[a, b] over the
// columns b owned by subdomain s, in column order.  A row whose neighbours
// all lie in one subdomain has AZ_i[a, s] = 0 in exact arithmetic (the
// stiffness rows sum to zero away from the boundary); such sums, which
// cancel to within 64 u of their terms' magnitudes in every input term, are
// left out, so only rows at an interface or the Dirichlet boundary remain.
void build_az(sg_amg* a, const sg_op* op, const std::vector<int32_t>& owner, hipStream_t s) {
    const int n = op->n, L = op->L, P = op->P, ns = a->n_sub;
    // E_s [L_in x P] FP64 must fit the LDS of one work-group; otherwise the
    // cycle keeps forming the residual with a matvec
    if ((size_t)L * P * sizeof(double) > 64 * 1024) return;
    std::vector<double> vals((size_t)op->nnz * L);
    op->vals.download(vals.data(), vals.size(), s);
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int32_t> rows, ptr(1, 0), col;
    std::vector<double> val;
    std::vector<int32_t> subs;
    std::vector<double> acc, sab;
    for (int r = 0; r < n; ++r) {
        subs.clear();
        for (int e = op->h_rowptr[r]; e < op->h_rowptr[r + 1]; ++e) {
            const int sd = owner[op->h_col[e]];
            if (std::find(subs.begin(), subs.end(), sd) == subs.end()) subs.push_back(sd);
        }
        std::sort(subs.begin(), subs.end());
        const size_t before = col.size();
        for (int sd : subs) {
            acc.assign(L, 0.0);
            sab.assign(L, 0.0);
            for (int e = op->h_rowptr[r]; e < op->h_rowptr[r + 1]; ++e) {
                if (owner[op->h_col[e]] != sd) continue;
                for (int i = 0; i < L; ++i) {
                    acc[i] += vals[(size_t)e * L + i];
                    sab[i] += std::fabs(vals[(size_t)e * L + i]);
                }
            }
            bool keep = false;
            for (int i = 0; i < L && !keep; ++i)
                keep = std::fabs(acc[i]) > 64.0 * 1.1102230246251565e-16 * sab[i];
            if (!keep) continue;
            col.push_back(sd);
            val.insert(val.end(), acc.begin(), acc.end());
        }
        if (col.size() > before) {
            rows.push_back(r);
            ptr.push_back((int32_t)col.size());
        }
    }
    const sg_basis& B = op->basis;
    std::vector<int32_t> order(B.T);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::make_tuple(B.tk[x], B.ti[x], B.tj[x]) < std::make_tuple(B.tk[y], B.ti[y], B.tj[y]);
    });
    // ranges of the (k, i) pairs: kiptr[k L + i] .. kiptr[k L + i + 1]
    std::vector<int32_t> kiptr((size_t)P * L + 1, 0), tj(B.T);
    std::vector<double> tv(B.T);
    for (int q = 0; q < B.T; ++q) {
        const int t = order[q];
        tj[q] = B.tj[t];
        tv[q] = B.tv[t];
        kiptr[(size_t)B.tk[t] * L + B.ti[t] + 1]++;
    }
    for (size_t q = 0; q < (size_t)P * L; ++q) kiptr[q + 1] += kiptr[q];
    // entries grouped by subdomain (stable: row order within a subdomain)
    const int ne = (int)col.size();
    std::vector<int32_t> sptr(ns + 1, 0), rpos(ne);
    for (int e = 0; e < ne; ++e) sptr[col[e] + 1]++;
    for (int q = 0; q < ns; ++q) sptr[q + 1] += sptr[q];
    std::vector<double> sval((size_t)ne * L);
    {
        std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
        for (int e = 0; e < ne; ++e) {
            const int q = fill[col[e]]++;
            rpos[e] = q;
            std::copy(val.begin() + (size_t)e * L, val.begin() + (size_t)(e + 1) * L,
                      sval.begin() + (size_t)q * L);
        }
    }
    a->az_rows_n = (int)rows.size();
    a->az_rows.upload(rows, s);
    a->az_ptr.upload(ptr, s);
    a->az_rpos.upload(rpos, s);
    a->az_sptr.upload(sptr, s);
    a->az_sval.upload(sval, s);
    a->az_kptr.upload(kiptr, s);
    a->az_tj.upload(tj, s);
    a->az_tv.upload(tv, s);
    a->az_W.alloc((size_t)std::max(ne, 1) * P);
    a->az_op = op;
    HIP_OK(hipStreamSynchronize(s));
}

bool amg_is_geometric(const sg_amg* a) { return a->kind == SG_COARSE_GEOMETRIC; }
int amg_fine_n(const sg_amg* a) { return a->n; }

// Host part of the geometric coarse space on the N x N lattice with ratio r:
// P_0 (nested P1 interpolation, boundary coarse nodes dropped), P_0^T by
// coarse rows, and the Galerkin values C_i = P_0^T K_i P_0 with the mesh
// graph of the coarse lattice.  Every fine element lies in one coarse
// triangle, so the pattern of C_i is the coarse 7-point stencil; an
// off-diagonal entry whose every term cancels to rounding residue (|C| <=
// 1e-12 sum |contributions|, e.g. the hypotenuse pairs of a right-angled
// lattice, exactly zero in exact arithmetic) is left out, as the assembly
// leaves out zero-weight entries.
struct GeoHost {
    int Nc = 0, nc = 0;
    std::vector<int32_t> pcol, rptr, rcol, cptr, ccol;
    std::vector<double> pval, rval, cval;
    std::vector<int64_t> gptr;
    std::vector<int32_t> gcol;
};

void geometric_host(const sg_op* op, const std::vector<double>& vals, int r, GeoHost& g) {
    const int N = op->lattice_N, L = op->L;
    const int Nc = N / r, nf = op->n, nc = (Nc - 1) * (Nc - 1);
    SG_REQUIRE(nf == (N - 1) * (N - 1), "operator is not the lattice's");
    g.Nc = Nc; g.nc = nc;
    g.pcol.assign((size_t)3 * nf, 0);
    g.pval.assign((size_t)3 * nf, 0.0);
    for (int j = 1; j < N; ++j)
        for (int i = 1; i < N; ++i) {
            const int row = (j - 1) * (N - 1) + (i - 1);
            const int ci = i / r, cj = j / r;
            const double a = (double)(i % r) / r, b = (double)(j % r) / r;
            int cx[3], cy[3];
            double w[3];
            if (a >= b) {
                cx[0] = ci; cy[0] = cj; w[0] = 1.0 - a;
                cx[1] = ci + 1; cy[1] = cj; w[1] = a - b;
                cx[2] = ci + 1; cy[2] = cj + 1; w[2] = b;
            } else {
                cx[0] = ci; cy[0] = cj; w[0] = 1.0 - b;
                cx[1] = ci + 1; cy[1] = cj + 1; w[1] = a;
                cx[2] = ci; cy[2] = cj + 1; w[2] = b - a;
            }
            for (int q = 0; q < 3; ++q)
                if (w[q] != 0.0 && cx[q] > 0 && cx[q] < Nc && cy[q] > 0 && cy[q] < Nc) {
                    g.pcol[(size_t)3 * row + q] = (cy[q] - 1) * (Nc - 1) + (cx[q] - 1);
                    g.pval[(size_t)3 * row + q] = w[q];
                }
        }
    // P_0^T by coarse rows, fine rows ascending within a row
    g.rptr.assign(nc + 1, 0);
    for (size_t q = 0; q < g.pval.size(); ++q)
        if (g.pval[q] != 0.0) g.rptr[g.pcol[q] + 1]++;
    for (int I = 0; I < nc; ++I) g.rptr[I + 1] += g.rptr[I];
    g.rcol.resize(g.rptr[nc]);
    g.rval.resize(g.rptr[nc]);
    {
        std::vector<int32_t> fill(g.rptr.begin(), g.rptr.end() - 1);
        for (int a = 0; a < nf; ++a)
            for (int q = 0; q < 3; ++q) {
                const double w = g.pval[(size_t)3 * a + q];
                if (w == 0.0) continue;
                const int32_t at = fill[g.pcol[(size_t)3 * a + q]]++;
                g.rcol[at] = a;
                g.rval[at] = w;
            }
    }
    // Galerkin triple product into the 7 stencil slots of every coarse row:
    // (dx, dy) = (-1,-1), (0,-1), (-1,0), (0,0), (1,0), (0,1), (1,1), which is
    // also increasing column order
    static const int kDx[7] = {-1, 0, -1, 0, 1, 0, 1}, kDy[7] = {-1, -1, 0, 0, 0, 1, 1};
    static const int kSlot[3][3] = {{0, 1, -1}, {2, 3, 4}, {-1, 5, 6}};
    const int W = Nc - 1;
    std::vector<double> acc((size_t)nc * 7 * L, 0.0), sab((size_t)nc * 7 * L, 0.0);
    for (int a = 0; a < nf; ++a)
        for (int p = 0; p < 3; ++p) {
            const double wp = g.pval[(size_t)3 * a + p];
            if (wp == 0.0) continue;
            const int I = g.pcol[(size_t)3 * a + p];
            const int Ix = I % W, Iy = I / W;
            for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e) {
                const int b = op->h_col[e];
                const double* v = vals.data() + (size_t)e * L;
                for (int q = 0; q < 3; ++q) {
                    const double wq = g.pval[(size_t)3 * b + q];
                    if (wq == 0.0) continue;
                    const int J = g.pcol[(size_t)3 * b + q];
                    const int dx = J % W - Ix, dy = J / W - Iy;
                    SG_REQUIRE(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 &&
                                   kSlot[dy + 1][dx + 1] >= 0,
                               "operator couples nodes outside one coarse triangle");
                    const size_t base = ((size_t)I * 7 + kSlot[dy + 1][dx + 1]) * L;
                    const double w = wp * wq;
                    for (int l = 0; l < L; ++l) {
                        const double t = w * v[l];
                        acc[base + l] += t;
                        sab[base + l] += std::fabs(t);
                    }
                }
            }
        }
    g.cptr.assign(nc + 1, 0);
    g.gptr.assign(nc + 1, 0);
    for (int I = 0; I < nc; ++I) {
        const int Ix = I % W, Iy = I / W;
        for (int sl = 0; sl < 7; ++sl) {
            const int x = Ix + kDx[sl], y = Iy + kDy[sl];
            if (x < 0 || x >= W || y < 0 || y >= W) continue;
            const int J = y * W + x;
            if (sl != 3) g.gcol.push_back(J);
            const size_t base = ((size_t)I * 7 + sl) * L;
            bool keep = sl == 3;
            for (int l = 0; l < L && !keep; ++l)
                keep = std::fabs(acc[base + l]) > 1e-12 * sab[base + l];
            if (!keep) continue;
            g.ccol.push_back(J);
            g.cval.insert(g.cval.end(), acc.begin() + base, acc.begin() + base + L);
        }
        g.cptr[I + 1] = (int32_t)g.ccol.size();
        g.gptr[I + 1] = (int64_t)g.gcol.size();
    }
}

}  // namespace sg

extern "C" {

int amg_setup_geometric(const sg_op* op, int ratio, const int32_t* owner_c, int n_sub_c,
                        int overlap, sg_coarse_kind level_coarse, sg_prec prec, double rtol,
                        int max_its, sg_amg** out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && owner_c && out, "null argument");
        SG_REQUIRE(op->lattice_N > 0,
                   "the geometric coarse space needs an operator assembled on the N x N lattice");
        const int N = op->lattice_N;
        SG_REQUIRE(ratio >= 1 && N % ratio == 0 && N / ratio >= 2,
                   "ratio %d must divide N = %d and leave at least 2 coarse cells", ratio, N);
        SG_REQUIRE(level_coarse == SG_COARSE_NONE || level_coarse == SG_COARSE_MEAN_EXACT ||
                       level_coarse == SG_COARSE_AMG, "bad coarse kind for the coarse level");
        SG_REQUIRE(prec == SG_FP64 || prec == SG_FP32 || prec == SG_BF16, "bad precision");
        SG_REQUIRE(rtol > 0.0 && rtol < 1.0, "coarse rtol must be in (0, 1)");
        SG_REQUIRE(max_its >= 1 && max_its <= 1000, "coarse max_its=%d outside [1, 1000]",
                   max_its);
        SG_REQUIRE(op->P <= 256, "P=%d exceeds 256 in the restriction kernel", op->P);
        check_device(op->device);
        hipStream_t s = as_stream(stream);
        std::vector<double> vals((size_t)op->nnz * op->L);
        op->vals.download(vals.data(), vals.size(), s);
        HIP_OK(hipStreamSynchronize(s));
        GeoHost g;
        geometric_host(op, vals, ratio, g);
        vals.clear();
        vals.shrink_to_fit();

        auto a = std::make_unique<sg_amg>();
        a->device = op->device;
        a->kind = SG_COARSE_GEOMETRIC;
        a->prec = prec;
        a->n = op->n; a->n_sub = g.nc; a->P = op->P; a->L = op->L;
        a->ratio = ratio;
        a->h_nodes = {g.nc};
        a->h_agg0.assign(g.nc, -1);
        a->inner_rtol = rtol;
        a->g_max = max_its;
        a->g_restart = std::min(max_its, 64);
        a->gp_col.upload(g.pcol, s);
        a->gp_val.upload(g.pval, s);
        a->gr_ptr.upload(g.rptr, s);
        a->gr_col.upload(g.rcol, s);
        a->gr_val.upload(g.rval, s);
        a->gop = make_csr_op(op->basis, g.nc, g.cptr, g.ccol, g.cval, g.gptr, g.gcol, s);
        int rc = ras_setup(a->gop, owner_c, n_sub_c, overlap, prec, &a->gras, stream);
        if (rc != SG_OK) SG_THROW(rc, "coarse-level RAS: %s", sg_last_error());
        // the coarse problem is small and its kernels latency-bound: time the
        // RAS apply paths and the staged matvec's shapes once and keep the
        // fastest (every path computes the same operator up to rounding)
        rc = ras_autotune(a->gras, 5, nullptr, stream);
        if (rc != SG_OK) SG_THROW(rc, "coarse-level RAS autotune: %s", sg_last_error());
        double mv_ms[3];
        rc = sg_matvec_autotune(a->gop, 10, mv_ms, stream);
        if (rc != SG_OK && rc != SG_ERR_UNSUPPORTED)
            SG_THROW(rc, "coarse-level matvec autotune: %s", sg_last_error());
        if (level_coarse != SG_COARSE_NONE) {
            rc = amg_setup(a->gop, a->gras, level_coarse, prec, &a->gamg, stream);
            if (rc != SG_OK) SG_THROW(rc, "coarse-level coarse solver: %s", sg_last_error());
        }
        a->gws.alloc(fgmres_ws_np(g.nc, op->P, a->gamg, a->g_restart));
        LinOp A;
        A.kron = a->gop; A.n = g.nc; A.P = op->P;
        double rho = 0.0;
        a->g_omega = smoother_damping_core(A, a->gras, 15, a->gws.p, a->gws.n, s, &rho);
        HIP_OK(hipStreamSynchronize(s));
        *out = a.release();
        return SG_OK;
    });
}

/* host outputs (any may be NULL): the coarse problem of a geometric coarse
 * space: its unknowns, the entries of its pattern, its smoother damping. */
int amg_geometric_info(const sg_amg* a, int* n_c, int64_t* nnz_c, double* omega_c) {
    return guarded([&]() -> int {
        SG_REQUIRE(a != nullptr, "amg is NULL");
        SG_REQUIRE(a->kind == SG_COARSE_GEOMETRIC, "not a geometric coarse space");
        if (n_c) *n_c = a->n_sub;
        if (nnz_c) *nnz_c = a->gop->nnz;
        if (omega_c) *omega_c = a->g_omega;
        return SG_OK;
    });
}

/* The coarse operator of a geometric coarse space (owned by `a`; valid until
 * sg_destroy_amg(a)), e.g. for sg_op_export. */
const sg_op* amg_geometric_op(const sg_amg* a) {
    return (a && a->kind == SG_COARSE_GEOMETRIC) ? a->gop : nullptr;
}

int amg_setup(const sg_op* op, const sg_ras* ras, sg_coarse_kind kind, sg_prec prec,
              sg_amg** out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && ras && out, "null argument");
        SG_REQUIRE(kind == SG_COARSE_MEAN_EXACT || kind == SG_COARSE_AMG, "bad coarse kind");
        SG_REQUIRE(prec == SG_FP64 || prec == SG_FP32 || prec == SG_BF16, "bad precision");
        SG_REQUIRE(op->P <= kBlk, "P=%d exceeds %d in the coarse solver", op->P, kBlk);
        check_device(op->device);
        SG_REQUIRE(ras_device(ras) == op->device, "ras and op on different devices");
        hipStream_t s = as_stream(stream);
        const int n = op->n, P = op->P, L = op->L;
        const int ns = ras_nsub(ras);
        const std::vector<int32_t>& owner = ras_owner(ras);
        SG_REQUIRE((int)owner.size() == n, "ras built for another operator");
        SG_REQUIRE(256 / P >= 1, "P too large for the restriction kernel");
        auto a = std::make_unique<sg_amg>();
        a->device = op->device; a->kind = kind; a->prec = prec;
        a->n = n; a->n_sub = ns; a->P = P; a->L = L;

        amg_common_setup(a.get(), owner, s);
        a->afact.upload(op->h_afact, s);
        // coarse pattern and the fine entries of every coarse entry
        std::vector<std::pair<int64_t, int64_t>> keyed;   // (coarse key, fine entry)
        keyed.reserve(op->nnz);
        for (int r = 0; r < n; ++r)
            for (int e = op->h_rowptr[r]; e < op->h_rowptr[r + 1]; ++e)
                keyed.push_back({(int64_t)owner[r] * ns + owner[op->h_col[e]], (int64_t)e});
        std::stable_sort(keyed.begin(), keyed.end(),
                         [](const auto& x, const auto& y) { return x.first < y.first; });
        std::vector<int32_t> cptr_row(ns + 1, 0), ccol;
        std::vector<int64_t> cptr(1, 0), cfine;
        for (size_t q = 0; q < keyed.size();) {
            size_t q1 = q;
            while (q1 < keyed.size() && keyed[q1].first == keyed[q].first) cfine.push_back(keyed[q1++].second);
            ccol.push_back((int32_t)(keyed[q].first % ns));
            cptr_row[keyed[q].first / ns + 1]++;
            cptr.push_back((int64_t)cfine.size());
            q = q1;
        }
        for (int q = 0; q < ns; ++q) cptr_row[q + 1] += cptr_row[q];
        const int64_t nce = (int64_t)ccol.size();
        DevBuf<int64_t> d_cptr, d_cfine;
        DevBuf<double> d_C(nce * L);
        d_cptr.upload(cptr, s);
        d_cfine.upload(cfine, s);
        coarse_entries_kernel<<<(unsigned)((nce * L + 255) / 256), 256, 0, s>>>(
            nce, L, d_cptr.p, d_cfine.p, op->vals.p, d_C.p);
        HIP_LAUNCH_OK();
        std::vector<double> C((size_t)nce * L);
        d_C.download(C.data(), C.size(), s);
        HIP_OK(hipStreamSynchronize(s));
        if (op->fixed_values) build_az(a.get(), op, owner, s);

        if (kind == SG_COARSE_MEAN_EXACT) {
            std::vector<double> C0((size_t)ns * ns, 0.0);
            for (int r = 0; r < ns; ++r)
                for (int q = cptr_row[r]; q < cptr_row[r + 1]; ++q)
                    C0[(size_t)r * ns + ccol[q]] = C[(size_t)q * L];
            invert_dense(C0, ns);
            a->c0inv.upload(C0, s);
            a->h_nodes = {ns};
            a->h_agg0.assign(ns, -1);
            HIP_OK(hipStreamSynchronize(s));
            *out = a.release();
            return SG_OK;
        }

        // level 0 block matrix: block (s,t) = sum_i C_i[s,t] G_i
        const sg_basis& B = op->basis;
        Bsr A;
        A.nr = A.nc = ns; A.P = P;
        A.ptr = cptr_row;
        A.col = ccol;
        A.val.assign((size_t)nce * P * P, 0.0);
        for (int64_t q = 0; q < nce; ++q) {
            double* blk = A.blk(q);
            for (int t = 0; t < B.T; ++t)
                blk[(size_t)B.tk[t] * P + B.tj[t]] += C[(size_t)q * L + B.ti[t]] * B.tv[t];
        }
        amg_build_hierarchy(a.get(), std::move(A), s);
        HIP_OK(hipStreamSynchronize(s));
        *out = a.release();
        return SG_OK;
    });
}

int amg_info(const sg_amg* a, int* n_levels, int32_t* nodes_per_level, int32_t* agg) {
    return guarded([&]() -> int {
        SG_REQUIRE(a != nullptr, "amg is NULL");
        if (n_levels) *n_levels = (int)a->h_nodes.size();
        if (nodes_per_level)
            for (size_t l = 0; l < a->h_nodes.size(); ++l) nodes_per_level[l] = a->h_nodes[l];
        if (agg) std::memcpy(agg, a->h_agg0.data(), a->n_sub * sizeof(int32_t));
        return SG_OK;
    });
}

int amg_level_blocks(const sg_amg* a, int level, int64_t* a_blocks, int64_t* p_blocks,
                     int64_t* r_blocks) {
    return guarded([&]() -> int {
        SG_REQUIRE(a != nullptr, "amg is NULL");
        SG_REQUIRE(level >= 0 && level < (int)a->lev.size(), "level %d out of range (%zu levels)",
                   level, a->lev.size());
        const AmgLevel& L = a->lev[level];
        const bool coarsest = level == (int)a->lev.size() - 1;
        if (a_blocks) *a_blocks = coarsest ? (int64_t)L.nn * L.nn : (int64_t)L.a_col.n;
        if (p_blocks) *p_blocks = coarsest ? 0 : (int64_t)L.p_col.n;
        if (r_blocks) *r_blocks = coarsest ? 0 : (int64_t)L.r_col.n;
        return SG_OK;
    });
}

int amg_vcycle(const sg_amg* a, const double* b_c, double* x_c, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(a && b_c && x_c, "null argument");
        SG_REQUIRE(b_c != x_c, "b_c and x_c must not alias");
        check_device(a->device);
        coarse_solve_base(a, b_c, x_c, as_stream(stream));
        return SG_OK;
    });
}

int amg_set_inner(sg_amg* a, sg_inner_kind inner, double rtol, int max_its) {
    return guarded([&]() -> int {
        SG_REQUIRE(a != nullptr, "amg is NULL");
        SG_REQUIRE(inner == SG_INNER_NONE || inner == SG_INNER_GMRES_AMG ||
                       inner == SG_INNER_GMRES_BJ, "bad inner kind %d", (int)inner);
        if (inner == SG_INNER_NONE) {
            a->inner = SG_INNER_NONE;
            return SG_OK;
        }
        SG_REQUIRE(a->kind == SG_COARSE_AMG, "an inner Krylov solve needs an SG_COARSE_AMG hierarchy");
        SG_REQUIRE(rtol > 0.0 && rtol < 1.0, "inner rtol must be in (0, 1)");
        SG_REQUIRE(max_its >= 1 && max_its <= kMaxInnerIts, "inner max_its=%d outside [1, %d]",
                   max_its, kMaxInnerIts);
        check_device(a->device);
        const int64_t N = (int64_t)a->n_sub * a->P;
        const int64_t ld = (N + 31) / 32 * 32;
        if (a->inner_max != max_its || a->inner_ld != ld) {
            // the last inner solve's combination may still be reading the basis
            HIP_OK(hipDeviceSynchronize());
            a->iV.alloc((size_t)(max_its + 1) * ld);
            a->iZ.alloc((size_t)max_its * ld);
            a->iw.alloc((size_t)ld);
            a->ismall.alloc((size_t)(max_its + 1) * max_its + 6 * (size_t)(max_its + 1) + 4);
        }
        if (!a->ipin) HIP_OK(hipHostMalloc(&a->ipin, 2 * sizeof(double), hipHostMallocDefault));
        a->inner = inner;
        a->inner_rtol = rtol;
        a->inner_max = max_its;
        a->inner_ld = ld;
        return SG_OK;
    });
}

int amg_inner_stats(const sg_amg* a, int64_t* calls, int64_t* its, int* last_its) {
    return guarded([&]() -> int {
        SG_REQUIRE(a != nullptr, "amg is NULL");
        if (calls) *calls = a->inner_calls;
        if (its) *its = a->inner_its;
        if (last_its) *last_its = a->inner_last;
        return SG_OK;
    });
}

int amg_coarse_solve(const sg_amg* a, const double* b_c, double* x_c, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(a && b_c && x_c, "null argument");
        SG_REQUIRE(b_c != x_c, "b_c and x_c must not alias");
        check_device(a->device);
        coarse_solve(a, b_c, x_c, as_stream(stream));
        return SG_OK;
    });
}

int sg_coarse_restrict(const sg_amg* a, const double* R, double* r_c, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(a && R && r_c, "null argument");
        check_device(a->device);
        coarse_restrict(a, R, r_c, as_stream(stream));
        return SG_OK;
    });
}

int sg_coarse_prolong_add(const sg_amg* a, const double* e_c, double* Y, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(a && e_c && Y, "null argument");
        check_device(a->device);
        coarse_prolong_add(a, e_c, Y, as_stream(stream));
        return SG_OK;
    });
}

void sg_destroy_amg(sg_amg* a) {
    sg::graph_cache_purge(a);
    delete a;
}

}  // extern "C"
