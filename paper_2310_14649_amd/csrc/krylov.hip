// Two-grid preconditioner application (Eq. RAS_2L as the cycle the text
// describes) and right-preconditioned flexible GMRES(m) in FP64 (the outer
// solver of Secs. 3-4).
//
// Arnoldi orthogonalisation, selectable: modified Gram-Schmidt (one kernel
// per basis vector: it reduces the previous dot product's partials, updates
// w and forms the next partials in the same pass), classical Gram-Schmidt
// with one conditional reorthogonalisation pass (when the first removed more
// than 1 - 1/sqrt(2) of ||w||), or single-pass classical Gram-Schmidt; the
// classical variants read the basis twice per pass instead of streaming w
// once per basis vector.  All reductions sum per-block partials in a fixed
// order, so results are bitwise reproducible.  The Hessenberg column, the Givens rotations and the residual
// estimate stay on the device; the host reads one scalar per iteration.
#include "common.hpp"

#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace sg {
namespace {

constexpr int kVT = 256;      // threads per vector block

inline int red_blocks(int64_t N) {
    int64_t b = (N + kVT * 4 - 1) / (kVT * 4);
    if (b < 1) b = 1;
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)b;
}

__device__ inline double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = kVT / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of nb partials in a fixed order (identical in every block).
__device__ inline double reduce_partials(const double* part, int nb, double* sh) {
    double a = 0.0;
    for (int q = threadIdx.x; q < nb; q += kVT) a += part[q];
    return block_sum(a, sh);
}

__global__ __launch_bounds__(kVT) void dot_partial_kernel(int64_t N, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          double* __restrict__ part) {
    __shared__ double sh[kVT];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVT)
        a = fma(x[i], y[i], a);
    double s = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kVT) void reduce_kernel(int nb, const double* __restrict__ part,
                                                     double* __restrict__ out) {
    __shared__ double sh[kVT];
    double s = reduce_partials(part, nb, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// w -= h v_i with h = sum(part_in); part_out = partial <w, v_next> (or <w,w>).
__global__ __launch_bounds__(kVT) void mgs_kernel(int64_t N, int nb, double* __restrict__ w,
                                                  const double* __restrict__ vi,
                                                  const double* __restrict__ vnext,
                                                  const double* __restrict__ part_in,
                                                  double* __restrict__ part_out,
                                                  double* __restrict__ hslot) {
    __shared__ double sh[kVT];
    const double h = reduce_partials(part_in, nb, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) hslot[0] = h;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVT) {
        const double wi = fma(-h, vi[i], w[i]);
        w[i] = wi;
        a = fma(wi, vnext ? vnext[i] : wi, a);
    }
    double s = block_sum(a, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

// ---- classical Gram-Schmidt with one conditional reorthogonalisation
// (Daniel-Gragg-Kaufman-Stewart criterion: a second pass when the first
// removes more than 1 - 1/sqrt(2) of ||w||).  Per pass: one kernel forms
// the partial sums of <w, v_i> for all i (and <w, w>), one reduces them in a
// fixed order, one subtracts sum_i h_i v_i; so w and the basis are read
// twice per pass instead of once per basis vector.
constexpr int kCgsIB = 16;      // basis vectors per work-group column of the dot kernel

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// part[i * nb + block] = partial <w, v_{i0+i}> (i < ni, this column's share)
// and, in column 0, part[ni * nb + block] = partial <w, w>.  Skipped unless
// *active (a null pointer means always).
__global__ __launch_bounds__(kVT) void cgs_dot_kernel(int64_t N, int nb, int ni, int64_t ldv,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ V,
                                                      double* __restrict__ part,
                                                      const double* __restrict__ active) {
    if (active && active[0] == 0.0) return;
    __shared__ double sh[kVT / 64][kCgsIB + 1];
    const int ib0 = blockIdx.y * kCgsIB;
    const int cnt = min(kCgsIB, ni - ib0);
    const bool with_ww = blockIdx.y == 0;
    double acc[kCgsIB + 1];
#pragma unroll
    for (int q = 0; q <= kCgsIB; ++q) acc[q] = 0.0;
    // pairs of elements through 16-byte loads (V's columns start 256-byte
    // aligned), an odd last element by the first thread
    const int64_t N2 = N >> 1;
    const double2* w2 = reinterpret_cast<const double2*>(w);
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N2; e += (int64_t)gridDim.x * kVT) {
        const double2 we = w2[e];
#pragma unroll
        for (int q = 0; q < kCgsIB; ++q)
            if (q < cnt) {
                const double2 v = reinterpret_cast<const double2*>(V + (size_t)(ib0 + q) * ldv)[e];
                acc[q] = fma(we.y, v.y, fma(we.x, v.x, acc[q]));
            }
        if (with_ww) acc[kCgsIB] = fma(we.y, we.y, fma(we.x, we.x, acc[kCgsIB]));
    }
    if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double we = w[N - 1];
#pragma unroll
        for (int q = 0; q < kCgsIB; ++q)
            if (q < cnt) acc[q] = fma(we, V[(size_t)(ib0 + q) * ldv + N - 1], acc[q]);
        if (with_ww) acc[kCgsIB] = fma(we, we, acc[kCgsIB]);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q <= kCgsIB; ++q) {
        const double t = wave_sum(acc[q]);
        if (lane == 0) sh[wv][q] = t;
    }
    __syncthreads();
    if (threadIdx.x <= kCgsIB) {
        const int q = threadIdx.x;
        double t = 0.0;
        for (int u = 0; u < kVT / 64; ++u) t += sh[u][q];
        if (q < cnt) part[(size_t)(ib0 + q) * nb + blockIdx.x] = t;
        if (q == kCgsIB && with_ww) part[(size_t)ni * nb + blockIdx.x] = t;
    }
}

// One work-group per coefficient: out[i] (+)= sum over blocks of part[i],
// fixed order.  i = ni is <w, w> (written to ww).  Skipped unless *active.
__global__ __launch_bounds__(kVT) void cgs_reduce_kernel(int nb, int ni, const double* __restrict__ part,
                                                         double* __restrict__ h, int accumulate,
                                                         double* __restrict__ ww,
                                                         const double* __restrict__ active) {
    if (active && active[0] == 0.0) return;
    __shared__ double sh[kVT];
    const int i = blockIdx.x;
    const double t = reduce_partials(part + (size_t)i * nb, nb, sh);
    if (threadIdx.x == 0) {
        if (i < ni) h[i] = accumulate ? h[i] + t : t;
        else ww[0] = t;
    }
}

// w -= sum_{i < ni} c_i v_i with c = h (first pass) or the correction of
// the second pass; part_out = partial <w, w>.  Skipped unless *active.
__global__ __launch_bounds__(kVT) void cgs_update_kernel(int64_t N, int ni, int64_t ldv,
                                                         double* __restrict__ w,
                                                         const double* __restrict__ V,
                                                         const double* __restrict__ c,
                                                         double* __restrict__ part_out,
                                                         const double* __restrict__ active) {
    if (active && active[0] == 0.0) return;
    __shared__ double cs[64];
    __shared__ double sh[kVT];
    for (int q = threadIdx.x; q < ni; q += kVT) cs[q] = c[q];
    __syncthreads();
    double a = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N; e += (int64_t)gridDim.x * kVT) {
        double we = w[e];
        for (int q = 0; q < ni; ++q) we = fma(-cs[q], V[(size_t)q * ldv + e], we);
        w[e] = we;
        a = fma(we, we, a);
    }
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

// ---- S Krylov directions per Gram-Schmidt pass (SG_ORTHO_CGS_BLOCK2..4).
// Block (j .. j+S-1): u_1 = A M v_j and u_{t+1} = A M u_t (the flexible
// direction of column j+t is M u_t), all projected against v_0..v_j in one
// pass over the basis, then orthonormalised among themselves by a Cholesky
// factorisation R of their Gram matrix (U = V_new R), repeated once on the
// new vectors where a diagonal of R keeps less than 1e-4 of its column's
// squared norm.  The directions are stored consecutively in V (slots j+1 ..
// j+S), with stride ldv.  part[(S q + t) nb + block] = partial <u_t, v_q>.
template <int S> struct BlockGS {
    static constexpr int kB = S == 2 ? 16 : (S == 3 ? 10 : 8);   // basis vectors per column
    static constexpr int NG = S * (S + 1) / 2;                   // Gram entries (t <= u)
};

template <int S>
__global__ __launch_bounds__(kVT) void cgsb_dot_kernel(int64_t N, int nb, int ni, int64_t ldv,
                                                       const double* __restrict__ U,
                                                       const double* __restrict__ V,
                                                       double* __restrict__ part) {
    constexpr int kB = BlockGS<S>::kB;
    __shared__ double sh[kVT / 64][S * kB];
    const int ib0 = blockIdx.y * kB;
    const int cnt = min(kB, ni - ib0);
    double a[kB][S];
#pragma unroll
    for (int q = 0; q < kB; ++q)
#pragma unroll
        for (int t = 0; t < S; ++t) a[q][t] = 0.0;
    const int64_t N2 = N >> 1;
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N2; e += (int64_t)gridDim.x * kVT) {
        double2 x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) x[t] = reinterpret_cast<const double2*>(U + (size_t)t * ldv)[e];
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (q < cnt) {
                const double2 v = reinterpret_cast<const double2*>(V + (size_t)(ib0 + q) * ldv)[e];
#pragma unroll
                for (int t = 0; t < S; ++t) a[q][t] = fma(x[t].y, v.y, fma(x[t].x, v.x, a[q][t]));
            }
    }
    if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (q < cnt) {
                const double v = V[(size_t)(ib0 + q) * ldv + N - 1];
#pragma unroll
                for (int t = 0; t < S; ++t) a[q][t] = fma(U[(size_t)t * ldv + N - 1], v, a[q][t]);
            }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kB; ++q)
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const double r = wave_sum(a[q][t]);
            if (lane == 0) sh[wv][S * q + t] = r;
        }
    __syncthreads();
    if (threadIdx.x < S * cnt) {
        const int r = threadIdx.x;
        double t = 0.0;
        for (int u = 0; u < kVT / 64; ++u) t += sh[u][r];
        part[(size_t)(S * ib0 + r) * nb + blockIdx.x] = t;
    }
}

// Block r < S ni reduces coefficient r: c_t[q], q = r / S, t = r % S, into
// column j + t of the Hessenberg (column-major, leading dimension ldh).
template <int S>
__global__ __launch_bounds__(kVT) void cgsb_reduce_kernel(int nb, const double* __restrict__ part,
                                                          double* __restrict__ hj, int ldh) {
    __shared__ double sh[kVT];
    const int r = blockIdx.x;
    const double t = reduce_partials(part + (size_t)r * nb, nb, sh);
    if (threadIdx.x == 0) hj[(size_t)(r % S) * ldh + r / S] = t;
}

// U_t -= sum_q c_t[q] v_q (one pass over the basis); part_out[g nb + block]
// = partial Gram entry g of the projected vectors (pairs t <= u in order).
// Each thread takes two consecutive entries per step (16-byte loads and
// stores; ldv is even and the vectors 16-byte aligned); the last entry of
// an odd N goes to thread 0 of block 0.
template <int S>
__global__ __launch_bounds__(kVT) void cgsb_update_kernel(int64_t N, int nb, int ni, int64_t ldv,
                                                          double* __restrict__ U,
                                                          const double* __restrict__ V,
                                                          const double* __restrict__ hj, int ldh,
                                                          double* __restrict__ part_out) {
    constexpr int NG = BlockGS<S>::NG;
    __shared__ double cs[S][64];
    __shared__ double sh[kVT];
    for (int q = threadIdx.x; q < ni; q += kVT)
#pragma unroll
        for (int t = 0; t < S; ++t) cs[t][q] = hj[(size_t)t * ldh + q];
    __syncthreads();
    double g[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] = 0.0;
    auto gram = [&](const double* x) {
        int k = 0;
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int u = t; u < S; ++u) {
                g[k] = fma(x[t], x[u], g[k]);
                ++k;
            }
    };
    const int64_t N2 = N >> 1;
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N2; e += (int64_t)gridDim.x * kVT) {
        double x0[S], x1[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const double2 u2 = reinterpret_cast<const double2*>(U + (size_t)t * ldv)[e];
            x0[t] = u2.x;
            x1[t] = u2.y;
        }
#pragma unroll 4
        for (int q = 0; q < ni; ++q) {
            const double2 v = reinterpret_cast<const double2*>(V + (size_t)q * ldv)[e];
#pragma unroll
            for (int t = 0; t < S; ++t) {
                x0[t] = fma(-cs[t][q], v.x, x0[t]);
                x1[t] = fma(-cs[t][q], v.y, x1[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < S; ++t)
            reinterpret_cast<double2*>(U + (size_t)t * ldv)[e] = make_double2(x0[t], x1[t]);
        gram(x0);
        gram(x1);
    }
    if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) x[t] = U[(size_t)t * ldv + N - 1];
        for (int q = 0; q < ni; ++q) {
            const double v = V[(size_t)q * ldv + N - 1];
#pragma unroll
            for (int t = 0; t < S; ++t) x[t] = fma(-cs[t][q], v, x[t]);
        }
#pragma unroll
        for (int t = 0; t < S; ++t) U[(size_t)t * ldv + N - 1] = x[t];
        gram(x);
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const double r = block_sum(g[q], sh);
        if (threadIdx.x == 0) part_out[(size_t)q * nb + blockIdx.x] = r;
    }
}

// Cholesky factor of the S x S Gram matrix reduced from part (entries t <= u
// in order).  Returns the index of the first direction that broke down (its
// pivot not positive) or S; R[t][u] for t <= u, zero past a breakdown.
// *weak: a pivot kept less than 1e-4 of its column's diagonal.
template <int S>
__device__ inline int block_chol(const double* part, int nb, double* sh, double (&R)[S][S],
                                 bool* weak) {
    double G[S][S];
    int k = 0;
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
        for (int u = t; u < S; ++u) {
            G[t][u] = reduce_partials(part + (size_t)(k++) * nb, nb, sh);
            G[u][t] = G[t][u];
        }
    int bad = S;
    *weak = false;
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
        for (int u = 0; u < S; ++u) R[t][u] = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
        if (bad < S) break;
        double d = G[t][t];
#pragma unroll
        for (int q = 0; q < t; ++q) d -= R[q][t] * R[q][t];
        if (!(d > 0.0)) { bad = t; break; }
        if (d < 1e-4 * G[t][t]) *weak = true;
        R[t][t] = sqrt(d);
#pragma unroll
        for (int u = t + 1; u < S; ++u) {
            double o = G[t][u];
#pragma unroll
            for (int q = 0; q < t; ++q) o -= R[q][t] * R[q][u];
            R[t][u] = o / R[t][t];
        }
    }
    return bad;
}

// U = V_new R: V_new = U R^{-1} in place (forward substitution per entry);
// H(j+1+q, j+t) = R[q][t]; flag = 1 + (first direction that broke down), 0
// if none; gate = 1 where a pivot was weak (a second factorisation follows).
template <int S>
__global__ __launch_bounds__(kVT) void block_qr_kernel(int64_t N, int nb, int64_t ldv,
                                                       double* __restrict__ U,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ hj, int ldh, int j,
                                                       double* __restrict__ flag,
                                                       double* __restrict__ gate) {
    __shared__ double sh[kVT];
    double R[S][S];
    bool weak;
    const int bad = block_chol<S>(part, nb, sh, R, &weak);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int q = 0; q <= t; ++q) hj[(size_t)t * ldh + j + 1 + q] = R[q][t];
        flag[0] = bad < S ? (double)(bad + 1) : 0.0;
        gate[0] = (bad == S && weak) ? 1.0 : 0.0;
    }
    double inv[S];
#pragma unroll
    for (int t = 0; t < S; ++t) inv[t] = R[t][t] > 0.0 ? 1.0 / R[t][t] : 0.0;
    auto solve = [&](double* x) {
#pragma unroll
        for (int t = 0; t < S; ++t) {
            double y = x[t];
#pragma unroll
            for (int q = 0; q < t; ++q) y = fma(-R[q][t], x[q], y);
            x[t] = y * inv[t];
        }
    };
    // two consecutive entries per thread and step, as in cgsb_update_kernel
    const int64_t N2 = N >> 1;
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N2; e += (int64_t)gridDim.x * kVT) {
        double x0[S], x1[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const double2 u2 = reinterpret_cast<const double2*>(U + (size_t)t * ldv)[e];
            x0[t] = u2.x;
            x1[t] = u2.y;
        }
        solve(x0);
        solve(x1);
#pragma unroll
        for (int t = 0; t < S; ++t)
            reinterpret_cast<double2*>(U + (size_t)t * ldv)[e] = make_double2(x0[t], x1[t]);
    }
    if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) x[t] = U[(size_t)t * ldv + N - 1];
        solve(x);
#pragma unroll
        for (int t = 0; t < S; ++t) U[(size_t)t * ldv + N - 1] = x[t];
    }
}

// Where the gate is set: the Gram partials of the new vectors ...
template <int S>
__global__ __launch_bounds__(kVT) void gated_gram_kernel(int64_t N, int nb, int64_t ldv,
                                                         const double* __restrict__ U,
                                                         double* __restrict__ part,
                                                         const double* __restrict__ gate) {
    if (gate[0] == 0.0) return;
    constexpr int NG = BlockGS<S>::NG;
    __shared__ double sh[kVT];
    double g[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N; e += (int64_t)gridDim.x * kVT) {
        double x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) x[t] = U[(size_t)t * ldv + e];
        int k = 0;
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int u = t; u < S; ++u) {
                g[k] = fma(x[t], x[u], g[k]);
                ++k;
            }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const double r = block_sum(g[q], sh);
        if (threadIdx.x == 0) part[(size_t)q * nb + blockIdx.x] = r;
    }
}

// ... and a second factorisation R2: V = V R2^{-1}, H's block R <- R2 R.
template <int S>
__global__ __launch_bounds__(kVT) void gated_requr_kernel(int64_t N, int nb, int64_t ldv,
                                                          double* __restrict__ U,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ hj, int ldh,
                                                          int j, const double* __restrict__ gate) {
    if (gate[0] == 0.0) return;
    __shared__ double sh[kVT];
    double R2[S][S];
    bool weak;
    const int bad = block_chol<S>(part, nb, sh, R2, &weak);
    if (bad < S) return;     // past the gate the new vectors are independent
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double R[S][S];
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int q = 0; q < S; ++q) R[q][t] = q <= t ? hj[(size_t)t * ldh + j + 1 + q] : 0.0;
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int q = 0; q <= t; ++q) {
                double a = 0.0;
#pragma unroll
                for (int k = q; k <= t; ++k) a = fma(R2[q][k], R[k][t], a);
                hj[(size_t)t * ldh + j + 1 + q] = a;
            }
    }
    double inv[S];
#pragma unroll
    for (int t = 0; t < S; ++t) inv[t] = 1.0 / R2[t][t];
    for (int64_t e = (int64_t)blockIdx.x * kVT + threadIdx.x; e < N; e += (int64_t)gridDim.x * kVT) {
        double x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) x[t] = U[(size_t)t * ldv + e];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            double y = x[t];
#pragma unroll
            for (int q = 0; q < t; ++q) y = fma(-R2[q][t], x[q], y);
            x[t] = y * inv[t];
        }
#pragma unroll
        for (int t = 0; t < S; ++t) U[(size_t)t * ldv + e] = x[t];
    }
}

// Second pass wanted if ||w_after||^2 < ||w_before||^2 / 2.
__global__ __launch_bounds__(kVT) void dgks_kernel(int nb, const double* __restrict__ part_after,
                                                   const double* __restrict__ ww_before,
                                                   double* __restrict__ flag) {
    __shared__ double sh[kVT];
    const double after = reduce_partials(part_after, nb, sh);
    if (threadIdx.x == 0) flag[0] = (after < 0.5 * ww_before[0]) ? 1.0 : 0.0;
}

// h_{j+1,j} = ||w||, v_{j+1} = w / h  (or 0 and the breakdown flag).
__global__ __launch_bounds__(kVT) void normalize_kernel(int64_t N, int nb,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ vnext,
                                                        const double* __restrict__ part,
                                                        double* __restrict__ hslot,
                                                        double* __restrict__ flag) {
    __shared__ double sh[kVT];
    const double nrm = sqrt(reduce_partials(part, nb, sh));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hslot[0] = nrm;
        flag[0] = (nrm == 0.0) ? 1.0 : 0.0;
    }
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    // pairs through 16-byte accesses (both vectors start 256-byte aligned),
    // an odd last element by the first thread
    const int64_t N2 = N >> 1;
    const double2* w2 = reinterpret_cast<const double2*>(w);
    double2* v2 = reinterpret_cast<double2*>(vnext);
    for (int64_t i = (int64_t)blockIdx.x * kVT + threadIdx.x; i < N2; i += (int64_t)gridDim.x * kVT) {
        const double2 x = w2[i];
        v2[i] = make_double2(x.x * inv, x.y * inv);
    }
    if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) vnext[N - 1] = w[N - 1] * inv;
}

// Apply the previous rotations to column j, form rotation j, update g.
// ld = m+1 (column-major H).
__global__ void givens_kernel(int j, int ld, double* __restrict__ H, double* __restrict__ cs,
                              double* __restrict__ sn, double* __restrict__ g,
                              double* __restrict__ est) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* h = H + (size_t)j * ld;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    const double den = hypot(h[j], h[j + 1]);
    double c = 1.0, s = 0.0;
    if (den > 0.0) { c = h[j] / den; s = h[j + 1] / den; }
    cs[j] = c;
    sn[j] = s;
    h[j] = den;
    h[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    est[0] = fabs(g[j + 1]);
}

// y = R^{-1} g for the k x k upper-triangular rotated Hessenberg.
__global__ void trisolve_kernel(int k, int ld, const double* __restrict__ H,
                                const double* __restrict__ g, double* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double acc = g[i];
        for (int c = i + 1; c < k; ++c) acc -= H[(size_t)c * ld + i] * y[c];
        y[i] = acc / H[(size_t)i * ld + i];
    }
}

// x += sum_i y_i Z_i  (Z_i stored with stride ld >= N)
__global__ __launch_bounds__(kVT) void multi_axpy_kernel(int64_t N, int64_t ld, int k,
                                                         const double* __restrict__ y,
                                                         const double* __restrict__ Zb,
                                                         double* __restrict__ x) {
    __shared__ double ys[64];
    for (int q = threadIdx.x; q < k; q += kVT) ys[q] = y[q];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kVT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVT) {
        double acc = x[i];
        for (int q = 0; q < k; ++q) acc = fma(ys[q], Zb[(size_t)q * ld + i], acc);
        x[i] = acc;
    }
}

__global__ void scale_kernel(int64_t N, double a, const double* x, double* y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

__global__ void fill_kernel(int64_t N, double v, double* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

__global__ void init_cycle_kernel(int m1, double beta, double* __restrict__ g) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m1) g[i] = (i == 0) ? beta : 0.0;
}

inline unsigned grid_for(int64_t N) {
    int64_t b = (N + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

struct Vec {
    static void scale(int64_t N, double a, const double* x, double* y, hipStream_t s) {
        scale_kernel<<<grid_for(N), 256, 0, s>>>(N, a, x, y);
        HIP_LAUNCH_OK();
    }
    static void fill(int64_t N, double v, double* y, hipStream_t s) {
        fill_kernel<<<grid_for(N), 256, 0, s>>>(N, v, y);
        HIP_LAUNCH_OK();
    }
};


// workspace needed by the preconditioner: T [N], rc [ns*P], ec [ns*P]
size_t precond_ws_ns(int n, int P, int ns) {
    size_t N = (size_t)n * P;
    size_t b = align_up(N * 8);
    if (ns >= 0) b += 2 * align_up((size_t)ns * P * 8);
    return b;
}
size_t precond_ws_np(int n, int P, const sg_amg* amg) {
    return precond_ws_ns(n, P, amg ? amg_nsub(amg) : -1);
}
size_t precond_ws(const sg_op* op, const sg_amg* amg) { return precond_ws_np(op->n, op->P, amg); }

void precond_apply(const LinOp& A, const sg_ras* ras, const sg_amg* amg, double omega,
                   const double* R, double* Z, char* ws, hipStream_t s) {
    const int64_t N = (int64_t)A.n * A.P;
    if (!ras) {
        scale_kernel<<<grid_for(N), 256, 0, s>>>(N, 1.0, R, Z);
        HIP_LAUNCH_OK();
        return;
    }
    ras_apply_ex(ras, R, Z, omega, 0.0, s);                          // z1 = w M r
    if (!amg) return;
    double* T = reinterpret_cast<double*>(ws);
    double* rc = reinterpret_cast<double*>(ws + align_up(N * 8));
    double* ec = reinterpret_cast<double*>(ws + align_up(N * 8) +
                                           align_up((size_t)amg_nsub(amg) * A.P * 8));
    linop_apply(A, Z, T, -1.0, 1.0, R, s);                           // t = r - A z1
    coarse_restrict(amg, T, rc, s);
    coarse_solve(amg, rc, ec, s);
    // t = r - A z2 = (r - A z1) - (A Z) e_c: only interface and boundary rows
    // of A Z are non-zero for the Nicolaides space, so the update replaces a
    // matvec where the coarse space holds A Z.  Then z2 = z1 + Z e_c is not
    // needed before the last smoothing, whose fused store adds it where it can.
    const int32_t* cown = coarse_owner_dev(amg);
    if (cown && coarse_has_az(amg, A.kron) && ras_can_add_coarse(ras)) {
        coarse_residual_update(amg, A.kron, ec, T, s);
        ras_apply_ex(ras, T, Z, omega, 1.0, s, ec, cown);           // z = z1 + Q t + w M t2
        return;
    }
    coarse_prolong_add(amg, ec, Z, s);                               // z2 = z1 + Q t
    if (!coarse_residual_update(amg, A.kron, ec, T, s))
        linop_apply(A, Z, T, -1.0, 1.0, R, s);
    ras_apply_ex(ras, T, Z, omega, 1.0, s);                          // z = z2 + w M t
}

// ------------------------------------------------------------------ graphs
// Pinned host slots for the per-step residual estimates, two alternating,
// each behind its own event: the copy of one step's estimate does not hold up
// the launch of the next step.  The slots and events come from a per-device
// pool and go back to it (not freed) when the solve ends, after the stream
// has drained, so a solve nested in a preconditioner (the geometric coarse
// solve) does not allocate pinned memory on every call.
struct PinnedSlot {
    double* p = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
constexpr int kMaxPoolDevices = 64;
std::mutex g_pin_mu;
std::vector<PinnedSlot> g_pin_pool[kMaxPoolDevices];

struct PinnedEstimates {
    double* p = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t s;
    int dev;
    explicit PinnedEstimates(hipStream_t st) : s(st), dev(current_device()) {
        SG_REQUIRE(dev >= 0 && dev < kMaxPoolDevices, "device %d beyond the pinned pool", dev);
        {
            std::lock_guard<std::mutex> lk(g_pin_mu);
            if (!g_pin_pool[dev].empty()) {
                PinnedSlot sl = g_pin_pool[dev].back();
                g_pin_pool[dev].pop_back();
                p = sl.p;
                ev[0] = sl.ev[0];
                ev[1] = sl.ev[1];
                return;
            }
        }
        try {
            HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&p), 4 * sizeof(double),
                                 hipHostMallocDefault));
            for (auto& e : ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        } catch (...) {
            for (auto& e : ev)
                if (e) (void)hipEventDestroy(e);
            if (p) (void)hipHostFree(p);
            throw;
        }
    }
    ~PinnedEstimates() {
        (void)hipStreamSynchronize(s);
        std::lock_guard<std::mutex> lk(g_pin_mu);
        PinnedSlot sl;
        sl.p = p;
        sl.ev[0] = ev[0];
        sl.ev[1] = ev[1];
        g_pin_pool[dev].push_back(sl);
    }
    PinnedEstimates(const PinnedEstimates&) = delete;
    PinnedEstimates& operator=(const PinnedEstimates&) = delete;
};

struct GraphKey {
    const void *op, *ras, *amg, *ws;
    size_t ws_bytes;
    int m, j, ortho;
    uint64_t omega_bits;
    bool operator<(const GraphKey& o) const {
        return std::tie(op, ras, amg, ws, ws_bytes, m, j, ortho, omega_bits) <
               std::tie(o.op, o.ras, o.amg, o.ws, o.ws_bytes, o.m, o.j, o.ortho, o.omega_bits);
    }
};

std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t>& graph_cache() {
    static std::map<GraphKey, hipGraphExec_t> c;
    return c;
}
std::map<int, hipStream_t>& capture_streams() {
    static std::map<int, hipStream_t> c;
    return c;
}

hipStream_t capture_stream(int dev) {
    auto& cs = capture_streams();
    auto it = cs.find(dev);
    if (it != cs.end()) return it->second;
    hipStream_t st;
    HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    cs[dev] = st;
    return st;
}

}  // namespace

void graph_cache_purge(const void* handle) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto& c = graph_cache();
    for (auto it = c.begin(); it != c.end();) {
        if (it->first.op == handle || it->first.ras == handle || it->first.amg == handle) {
            (void)hipGraphExecDestroy(it->second);
            it = c.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace sg

namespace sg {

// Host-visible dot product (synchronous).
double host_dot(int64_t N, const double* x, const double* y, double* part, double* scal,
                hipStream_t s) {
    const int nb = red_blocks(N);
    dot_partial_kernel<<<nb, kVT, 0, s>>>(N, x, y, part);
    HIP_LAUNCH_OK();
    reduce_kernel<<<1, kVT, 0, s>>>(nb, part, scal);
    HIP_LAUNCH_OK();
    double h = 0.0;
    HIP_OK(hipMemcpyAsync(&h, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return h;
}

size_t fgmres_ws_ns(int n, int P, int ns, int restart) {
    const size_t N = (size_t)n * P;
    const size_t m = (size_t)restart;
    size_t b = align_up(N * 8) * (2 * m + 2);                 // V (m+1), Z (m), w
    b += precond_ws_ns(n, P, ns);
    b += 2 * align_up(kMaxRedBlocks * 8);                     // partial sums
    b += align_up((4 * m + 8) * kMaxRedBlocks * 8);           // Gram-Schmidt partials
    b += align_up((m + 1) * 8) + align_up(64);                // correction, flags
    b += align_up((m + 1) * m * 8) + 4 * align_up((m + 1) * 8) + align_up(64);
    // the damping estimate reuses the front of the workspace
    const size_t damp = 2 * align_up(N * 8) + align_up(kMaxRedBlocks * 8) + 256;
    return b > damp ? b : damp;
}

size_t fgmres_ws_np(int n, int P, const sg_amg* amg, int restart) {
    return fgmres_ws_ns(n, P, amg ? amg_nsub(amg) : -1, restart);
}

// Entry i of the power iteration's start: output i + 1 of the SplitMix64
// generator (Steele, Lea and Flood, OOPSLA 2014) from state 0, its top 53 bits
// as a uniform in [-1/2, 1/2).  A smooth start (all ones) holds too little of
// the oscillating top modes for 15 steps to find them.
__global__ __launch_bounds__(256) void power_start_kernel(int64_t N, double* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * 256) {
        uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        y[i] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
    }
}

// Power estimate of rho(M A) from the pseudo-random start; returns the
// smoother damping min(1, 1.8/rho).  ws: >= 2 vectors + partial sums.
double smoother_damping_core(const LinOp& A, const sg_ras* ras, int its, char* p, size_t ws_bytes,
                             hipStream_t s, double* rho_out) {
    const int64_t N = (int64_t)A.n * A.P;
    const size_t need = 2 * align_up(N * 8) + align_up(kMaxRedBlocks * 8) + 256;
    if (!p || ws_bytes < need)
        SG_THROW(SG_ERR_WORKSPACE, "damping workspace too small (%zu < %zu)", ws_bytes, need);
    double* v = reinterpret_cast<double*>(p);
    double* w = reinterpret_cast<double*>(p + align_up(N * 8));
    double* part = reinterpret_cast<double*>(p + 2 * align_up(N * 8));
    double* scal = reinterpret_cast<double*>(p + 2 * align_up(N * 8) + align_up(kMaxRedBlocks * 8));
    power_start_kernel<<<grid_for(N), 256, 0, s>>>(N, v);
    HIP_LAUNCH_OK();
    {
        const double n0 = std::sqrt(host_dot(N, v, v, part, scal, s));
        Vec::scale(N, 1.0 / n0, v, v, s);
    }
    double rho = 0.0;
    for (int it = 0; it < its; ++it) {
        linop_apply(A, v, w, 1.0, 0.0, nullptr, s);
        ras_apply_ex(ras, w, v, 1.0, 0.0, s);
        rho = std::sqrt(host_dot(N, v, v, part, scal, s));
        if (!(rho > 0.0) || !std::isfinite(rho)) SG_THROW(SG_ERR_NUMERIC, "power iteration broke down");
        Vec::scale(N, 1.0 / rho, v, v, s);
    }
    HIP_OK(hipStreamSynchronize(s));
    if (rho_out) *rho_out = rho;
    return std::min(1.0, 1.8 / rho);
}

// Flexible GMRES on any LinOp.  key_op identifies the operator in the graph
// cache (its handle or matrix storage).
int fgmres_core(const LinOp& A, const void* key_op, int device, const sg_ras* ras,
                const sg_amg* amg, const double* b, double* x, const sg_krylov_opts* opts,
                sg_krylov_stats* stats, void* ws, size_t ws_bytes, hipStream_t s) {
    SG_REQUIRE(b && x && opts, "null argument");
    SG_REQUIRE(b != x, "b and x must not alias");
    const int m = opts->restart;
    SG_REQUIRE(m >= 1 && m <= 64, "restart=%d outside [1,64]", m);
    SG_REQUIRE(opts->max_it >= 1, "max_it must be >= 1");
    SG_REQUIRE(opts->rtol > 0.0, "rtol must be > 0");
    SG_REQUIRE(opts->ortho >= SG_ORTHO_MGS && opts->ortho <= SG_ORTHO_CGS_BLOCK4,
               "bad orthogonalisation");
    const size_t need = fgmres_ws_np(A.n, A.P, amg, m);
    if (!ws || ws_bytes < need)
        SG_THROW(SG_ERR_WORKSPACE, "fgmres workspace too small (%zu < %zu)", ws_bytes, need);
    SG_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, "workspace must be 256-byte aligned");
    const int64_t N = (int64_t)A.n * A.P;
    const size_t vb = align_up(N * 8);
    char* p = reinterpret_cast<char*>(ws);
    double* V = reinterpret_cast<double*>(p);                         // (m+1) vectors
    double* Zb = reinterpret_cast<double*>(p + vb * (m + 1));         // m vectors
    double* w = reinterpret_cast<double*>(p + vb * (2 * m + 1));
    char* pws = p + vb * (2 * m + 2);
    char* q = pws + precond_ws_np(A.n, A.P, amg);
    double* part0 = reinterpret_cast<double*>(q); q += align_up(kMaxRedBlocks * 8);
    double* part1 = reinterpret_cast<double*>(q); q += align_up(kMaxRedBlocks * 8);
    double* gsp = reinterpret_cast<double*>(q); q += align_up((size_t)(4 * m + 8) * kMaxRedBlocks * 8);
    double* corr = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * 8);
    double* gsf = reinterpret_cast<double*>(q); q += align_up(64);   // ww_before, flag
    double* H = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * m * 8);
    double* cs = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * 8);
    double* sn = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * 8);
    double* g = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * 8);
    double* y = reinterpret_cast<double*>(q); q += align_up((size_t)(m + 1) * 8);
    double* scal = reinterpret_cast<double*>(q);                      // est, flag, dot
    double* part[2] = {part0, part1};
        const int nb = red_blocks(N);

        double omega = opts->omega;
        if (ras && !(omega > 0.0)) {
            double rho = 0.0;
            omega = smoother_damping_core(A, ras, 15, reinterpret_cast<char*>(ws), ws_bytes, s, &rho);
        }
        if (!(omega > 0.0)) omega = 1.0;

        auto t0 = std::chrono::steady_clock::now();
        const double bnorm = std::sqrt(host_dot(N, b, b, part0, scal + 2, s));
        int its = 0, restarts = 0, hist = 0;
        bool converged = false;
        auto push_hist = [&](double v) {
            if (stats && stats->history && hist < stats->history_cap) stats->history[hist] = v;
            ++hist;
        };
        double relres = 0.0;
        // One Arnoldi step: z_j = B v_j, w = A z_j, modified Gram-Schmidt
        // against v_0..v_j, v_{j+1} = w/||w||, Givens update of column j.
        auto arnoldi_step = [&](int j, hipStream_t st) {
            double* vj = V + (size_t)j * (vb / 8);
            double* zj = Zb + (size_t)j * (vb / 8);
            precond_apply(A, ras, amg, omega, vj, zj, pws, st);
            linop_apply(A, zj, w, 1.0, 0.0, nullptr, st);
            double* hcol = H + (size_t)j * (m + 1);
            const int ni = j + 1;
            const int64_t ldv = (int64_t)(vb / 8);
            double* part_w = part[0];                   // partial sums of ||w||^2 at the end
            if (opts->ortho == SG_ORTHO_MGS) {
                dot_partial_kernel<<<nb, kVT, 0, st>>>(N, w, V, part[0]);
                HIP_LAUNCH_OK();
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (size_t)i * (vb / 8);
                    const double* vn = (i < j) ? V + (size_t)(i + 1) * (vb / 8) : nullptr;
                    mgs_kernel<<<nb, kVT, 0, st>>>(N, nb, w, vi, vn, part[i & 1], part[(i + 1) & 1],
                                                   hcol + i);
                    HIP_LAUNCH_OK();
                }
                part_w = part[(j + 1) & 1];
            } else {
                const dim3 dgrid(nb, (ni + kCgsIB - 1) / kCgsIB);
                // first pass: h = V^T w, w -= V h
                cgs_dot_kernel<<<dgrid, kVT, 0, st>>>(N, nb, ni, ldv, w, V, gsp, nullptr);
                HIP_LAUNCH_OK();
                cgs_reduce_kernel<<<ni + 1, kVT, 0, st>>>(nb, ni, gsp, hcol, 0, gsf, nullptr);
                HIP_LAUNCH_OK();
                cgs_update_kernel<<<nb, kVT, 0, st>>>(N, ni, ldv, w, V, hcol, part[0], nullptr);
                HIP_LAUNCH_OK();
                if (opts->ortho == SG_ORTHO_CGS_DGKS) {
                    // second pass only where the first lost more than 1 - 1/sqrt(2) of ||w||
                    dgks_kernel<<<1, kVT, 0, st>>>(nb, part[0], gsf, gsf + 1);
                    HIP_LAUNCH_OK();
                    cgs_dot_kernel<<<dgrid, kVT, 0, st>>>(N, nb, ni, ldv, w, V, gsp, gsf + 1);
                    HIP_LAUNCH_OK();
                    cgs_reduce_kernel<<<ni, kVT, 0, st>>>(nb, ni, gsp, corr, 0, gsf + 2, gsf + 1);
                    HIP_LAUNCH_OK();
                    cgs_update_kernel<<<nb, kVT, 0, st>>>(N, ni, ldv, w, V, corr, part[0], gsf + 1);
                    HIP_LAUNCH_OK();
                    cgs_reduce_kernel<<<ni, kVT, 0, st>>>(nb, ni, gsp, hcol, 1, gsf + 2, gsf + 1);
                    HIP_LAUNCH_OK();
                }
            }
            double* vnext = V + (size_t)(j + 1) * (vb / 8);
            normalize_kernel<<<nb, kVT, 0, st>>>(N, nb, w, vnext, part_w, hcol + j + 1,
                                                 scal + 1);
            HIP_LAUNCH_OK();
            givens_kernel<<<1, 1, 0, st>>>(j, m + 1, H, cs, sn, g, scal);
            HIP_LAUNCH_OK();
        };
        // Block (j .. j+S-1) of SG_ORTHO_CGS_BLOCK2..4: z_j = M v_j, u_1 = A z_j,
        // z_{j+t} = M u_t, u_{t+1} = A z_{j+t}; the u projected against
        // v_0..v_j in one pass (coefficients into columns j .. j+S-1 of H),
        // then orthonormalised among themselves (Cholesky of their Gram
        // matrix) into v_{j+1} .. v_{j+S}, so that A z_i = V H(:, i) holds
        // for every column of the block.
        const int sblock = opts->ortho == SG_ORTHO_CGS_BLOCK2 ? 2
                         : opts->ortho == SG_ORTHO_CGS_BLOCK3 ? 3
                         : opts->ortho == SG_ORTHO_CGS_BLOCK4 ? 4 : 1;
        auto block_step = [&](int j, int S, hipStream_t st) {
            const int64_t ldv = (int64_t)(vb / 8);
            for (int t = 0; t < S; ++t) {
                const double* src = V + (size_t)(j + t) * ldv;     // v_j, then u_1 .. u_{S-1}
                double* zt = Zb + (size_t)(j + t) * ldv;
                precond_apply(A, ras, amg, omega, src, zt, pws, st);
                linop_apply(A, zt, V + (size_t)(j + t + 1) * ldv, 1.0, 0.0, nullptr, st);
            }
            const int ni = j + 1;
            double* U = V + (size_t)(j + 1) * ldv;
            double* hj = H + (size_t)j * (m + 1);
            const int ldh = m + 1;
            auto go = [&](auto tag) {
                constexpr int SB = decltype(tag)::value;
                const dim3 dgrid(nb, (ni + BlockGS<SB>::kB - 1) / BlockGS<SB>::kB);
                cgsb_dot_kernel<SB><<<dgrid, kVT, 0, st>>>(N, nb, ni, ldv, U, V, gsp);
                HIP_LAUNCH_OK();
                cgsb_reduce_kernel<SB><<<SB * ni, kVT, 0, st>>>(nb, gsp, hj, ldh);
                HIP_LAUNCH_OK();
                cgsb_update_kernel<SB><<<nb, kVT, 0, st>>>(N, nb, ni, ldv, U, V, hj, ldh, gsp);
                HIP_LAUNCH_OK();
                block_qr_kernel<SB><<<nb, kVT, 0, st>>>(N, nb, ldv, U, gsp, hj, ldh, j, scal + 1,
                                                         gsf + 3);
                HIP_LAUNCH_OK();
                gated_gram_kernel<SB><<<nb, kVT, 0, st>>>(N, nb, ldv, U, gsp, gsf + 3);
                HIP_LAUNCH_OK();
                gated_requr_kernel<SB><<<nb, kVT, 0, st>>>(N, nb, ldv, U, gsp, hj, ldh, j, gsf + 3);
                HIP_LAUNCH_OK();
            };
            if (S == 2) go(std::integral_constant<int, 2>{});
            else if (S == 3) go(std::integral_constant<int, 3>{});
            else go(std::integral_constant<int, 4>{});
            for (int t = 0; t < S; ++t) {
                givens_kernel<<<1, 1, 0, st>>>(j + t, m + 1, H, cs, sn, g, scal);
                HIP_LAUNCH_OK();
            }
        };
        // columns of the unit that starts at column j: a block of up to
        // sblock directions while they fit the cycle and the step budget
        auto width = [&](int j, int its_now) {
            return std::max(1, std::min(sblock, std::min(m - j, opts->max_it - its_now)));
        };
        if (bnorm == 0.0) {
            Vec::fill(N, 0.0, x, s);
            converged = true;
        } else {
            if (!std::isfinite(bnorm)) SG_THROW(SG_ERR_NUMERIC, "right-hand side is not finite");
            const double target = opts->rtol * bnorm;
            linop_apply(A, x, V, -1.0, 1.0, b, s);                        // r0 = b - A x0
            double beta = std::sqrt(host_dot(N, V, V, part0, scal + 2, s));
            if (!std::isfinite(beta)) SG_THROW(SG_ERR_NUMERIC, "initial residual is not finite");
            relres = beta / bnorm;
            push_hist(relres);
            if (beta <= target) converged = true;
            // one Arnoldi step (w = 1) or step pair (w = 2), from its captured
            // graph (captured on first use)
            auto launch_unit = [&](int j, int w) {
                auto run = [&](hipStream_t st) {
                    if (w >= 2) block_step(j, w, st);
                    else arnoldi_step(j, st);
                };
                if (!opts->use_graph || (amg && inner_active(amg))) {
                    run(s);
                    return;
                }
                hipGraphExec_t exec = nullptr;
                // a block's graph is keyed by its width, a single step by the
                // orthogonalisation it runs (blocks end with single-pass CGS)
                const int kortho = w >= 2 ? 100 + w
                                          : (sblock > 1 ? (int)SG_ORTHO_CGS : opts->ortho);
                GraphKey key{key_op, ras, amg, ws, ws_bytes, m, j, kortho, 0};
                std::memcpy(&key.omega_bits, &omega, sizeof(double));
                {
                    std::lock_guard<std::mutex> lk(g_graph_mu);
                    auto it = graph_cache().find(key);
                    if (it != graph_cache().end()) exec = it->second;
                }
                if (!exec) {
                    hipStream_t cst = capture_stream(device);
                    HIP_OK(hipStreamSynchronize(s));
                    HIP_OK(hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal));
                    try {
                        run(cst);
                    } catch (...) {
                        hipGraph_t bad = nullptr;
                        (void)hipStreamEndCapture(cst, &bad);
                        if (bad) (void)hipGraphDestroy(bad);
                        throw;
                    }
                    hipGraph_t graph = nullptr;
                    HIP_OK(hipStreamEndCapture(cst, &graph));
                    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    HIP_OK(ie);
                    std::lock_guard<std::mutex> lk(g_graph_mu);
                    graph_cache()[key] = exec;
                }
                HIP_OK(hipGraphLaunch(exec, s));
            };
            PinnedEstimates pin(s);
            while (!converged && its < opts->max_it) {
                init_cycle_kernel<<<1, 128, 0, s>>>(m + 1, beta, g);
                HIP_LAUNCH_OK();
                Vec::scale(N, 1.0 / beta, V, V, s);
                int jd = 0;
                int launched = -1;                  // first column of the unit in flight
                double est_prev[2] = {0.0, 0.0};   // estimates of the last two units
                int unit = 0;
                for (int j = 0; j < m;) {
                    const int w = width(j, its);
                    if (launched != j) launch_unit(j, w);
                    double* hb = pin.p + 2 * (unit & 1);
                    HIP_OK(hipMemcpyAsync(hb, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
                    HIP_OK(hipEventRecord(pin.ev[unit & 1], s));
                    // The next unit (one step, or a step pair) runs while the
                    // host reads this one's estimate.  A unit past convergence
                    // writes only columns from j + w on of H, g[j + w ..], and
                    // V, Z beyond the columns the update with j + w columns
                    // reads; it is not started where the last two estimates
                    // extrapolate to within 4 x the target (wasted work).
                    const int jn = j + w;
                    const bool near = unit >= 2 && est_prev[1] > 0.0 &&
                                      est_prev[0] * est_prev[0] / est_prev[1] <= 4.0 * target;
                    launched = -1;
                    if (jn < m && its + w < opts->max_it && !near) {
                        launch_unit(jn, width(jn, its + w));
                        launched = jn;
                    }
                    HIP_OK(hipEventSynchronize(pin.ev[unit & 1]));
                    const double hs[2] = {hb[0], hb[1]};
                    // a block whose direction t broke down keeps t + 1 columns
                    // (flag = t + 1; a single step's flag 1 keeps its column)
                    const int keep = (w >= 2 && hs[1] >= 1.0) ? (int)hs[1] : w;
                    its += keep;
                    jd = j + keep;
                    if (!std::isfinite(hs[0]))
                        SG_THROW(SG_ERR_NUMERIC, "Arnoldi produced a non-finite value");
                    relres = hs[0] / bnorm;
                    push_hist(relres);
                    if (hs[0] <= target || hs[1] != 0.0 || its >= opts->max_it) break;
                    est_prev[1] = est_prev[0];
                    est_prev[0] = hs[0];
                    ++unit;
                    j = jn;
                }
                trisolve_kernel<<<1, 1, 0, s>>>(jd, m + 1, H, g, y);
                HIP_LAUNCH_OK();
                multi_axpy_kernel<<<grid_for(N), kVT, 0, s>>>(N, (int64_t)(vb / 8), jd, y, Zb, x);
                HIP_LAUNCH_OK();
                linop_apply(A, x, V, -1.0, 1.0, b, s);                    // true residual
                beta = std::sqrt(host_dot(N, V, V, part0, scal + 2, s));
                relres = beta / bnorm;
                if (beta <= target) { converged = true; break; }
                if (!std::isfinite(beta)) SG_THROW(SG_ERR_NUMERIC, "residual is not finite");
                ++restarts;
            }
        }
        HIP_OK(hipStreamSynchronize(s));
        auto t1 = std::chrono::steady_clock::now();
        if (stats) {
            stats->iterations = its;
            stats->restarts = restarts;
            stats->converged = converged ? 1 : 0;
            stats->true_relres = relres;
            stats->omega = omega;
            stats->ms_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
            stats->history_len = hist < stats->history_cap ? hist : stats->history_cap;
        }
        return converged ? SG_OK : SG_NOT_CONVERGED;
}

// ------------------------------------------------- the no-allocation apply
// Scratch of sg_precond_apply_noalloc: the workspace of sg_precond_apply
// (T [n*P], then r_c and e_c [n_sub*P], each 256-byte aligned) in a
// file-scope device array.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is not a device
// address: kernels receive the address hipGetSymbolAddress returns for the
// current device, looked up once per device and cached here.
static __device__ __align__(256) char scratch[SG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

char* scratch_ptr() {
    const int dev = current_device();
    SG_REQUIRE(dev >= 0 && dev < kMaxScratchDevices, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SG_REQUIRE(p != nullptr, "no device address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace sg

using namespace sg;

extern "C" {

size_t sg_precond_workspace_bytes(const sg_op* op, const sg_amg* amg) {
    if (!op) return 0;
    return precond_ws(op, amg);
}

static void check_set(const sg_op* op, const sg_ras* ras, const sg_amg* amg) {
    SG_REQUIRE(op != nullptr, "op is NULL");
    check_device(op->device);
    if (ras) {
        SG_REQUIRE(ras_device(ras) == op->device, "ras on another device");
        SG_REQUIRE(ras_n(ras) == op->n, "ras built for another operator");
    }
    if (amg) {
        SG_REQUIRE(ras != nullptr, "a coarse solver needs the RAS smoother");
        SG_REQUIRE(amg_device(amg) == op->device, "amg on another device");
        if (amg_is_geometric(amg))
            SG_REQUIRE(amg_fine_n(amg) == op->n, "amg built for another operator");
        else
            SG_REQUIRE(amg_nsub(amg) == ras_nsub(ras), "amg and ras disagree on subdomains");
    }
}

static LinOp kron_op(const sg_op* op) {
    LinOp A;
    A.kron = op;
    A.n = op->n;
    A.P = op->P;
    return A;
}

int sg_precond_apply(const sg_op* op, const sg_ras* ras, const sg_amg* amg, double omega,
                     const double* R, double* Z, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&]() -> int {
        check_set(op, ras, amg);
        SG_REQUIRE(R && Z && R != Z, "R, Z must be distinct non-null");
        SG_REQUIRE(ras != nullptr, "ras is NULL");
        if (amg) {
            if (!ws || ws_bytes < precond_ws(op, amg))
                SG_THROW(SG_ERR_WORKSPACE, "precond workspace too small (%zu < %zu)", ws_bytes,
                         precond_ws(op, amg));
        }
        precond_apply(kron_op(op), ras, amg, omega, R, Z, reinterpret_cast<char*>(ws),
                      as_stream(stream));
        return SG_OK;
    });
}

int sg_precond_apply_noalloc(const sg_op* op, const sg_ras* ras, const sg_amg* amg,
                             double omega, const double* R, double* Z, void* stream) {
    return guarded([&]() -> int {
        check_set(op, ras, amg);
        SG_REQUIRE(R && Z && R != Z, "R, Z must be distinct non-null");
        SG_REQUIRE(ras != nullptr, "ras is NULL");
        char* ws = nullptr;
        if (amg) {
            const size_t need = precond_ws(op, amg);
            if (need > (size_t)SG_NOALLOC_SCRATCH_BYTES)
                SG_THROW(SG_ERR_WORKSPACE,
                         "sg_precond_apply_noalloc needs %zu bytes of scratch, the static "
                         "scratch holds %zu (use sg_precond_apply with a workspace)",
                         need, (size_t)SG_NOALLOC_SCRATCH_BYTES);
            ws = scratch_ptr();
        }
        // every scratch entry the cycle reads is written earlier in the same
        // call (t = r - A z1, r_c = Z^T t, e_c = coarse solve), so nothing left
        // by an earlier call is read and nothing needs clearing
        precond_apply(kron_op(op), ras, amg, omega, R, Z, ws, as_stream(stream));
        return SG_OK;
    });
}

int sg_smoother_damping(const sg_op* op, const sg_ras* ras, int its, double* rho_out,
                        double* omega_out, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&]() -> int {
        check_set(op, ras, nullptr);
        SG_REQUIRE(ras != nullptr, "ras is NULL");
        SG_REQUIRE(its >= 1, "its must be >= 1");
        double om = smoother_damping_core(kron_op(op), ras, its, reinterpret_cast<char*>(ws),
                                          ws_bytes, as_stream(stream), rho_out);
        if (omega_out) *omega_out = om;
        return SG_OK;
    });
}

int sg_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    int n = 0;
    for (auto& kv : graph_cache()) {
        (void)hipGraphExecDestroy(kv.second);
        ++n;
    }
    graph_cache().clear();
    return n;
}

size_t fgmres_workspace_bytes(const sg_op* op, const sg_amg* amg, int restart) {
    if (!op || restart < 1) return 0;
    return fgmres_ws_np(op->n, op->P, amg, restart);
}

int fgmres_solve(const sg_op* op, const sg_ras* ras, const sg_amg* amg, const double* b, double* x,
                 const sg_krylov_opts* opts, sg_krylov_stats* stats, void* ws, size_t ws_bytes,
                 void* stream) {
    return guarded([&]() -> int {
        check_set(op, ras, amg);
        return fgmres_core(kron_op(op), op, op->device, ras, amg, b, x, opts, stats, ws, ws_bytes,
                           as_stream(stream));
    });
}

}  // extern "C"
