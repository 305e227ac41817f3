// SG operator apply (Eq. Galerkin_L_exp in the vector-PDE layout of
// Eqs. linearVecPDE / Ajklinear):
//
//     Y[a, k] = sum_i sum_b K_i[a, b] sum_j m_ijk X[b, j]
//
// computed per tile of consecutive rows in two phases that share the LDS:
//   1. W[r][i][j] = sum_b K_i[a_r, b] X[b, j]   (sparse rows x dense n-by-P block;
//      the tile's CSR values are staged in LDS and broadcast to the P lanes
//      of a row, X rows are read coalesced along j)
//   2. Y[a_r, k] = sum over stored triples (i, j, k) of m_ijk W[r][i][j]
//      (the triple table of the operator sits in LDS, sorted by k).
// Only the non-zero triples are touched, so the contraction costs T flops
// per row instead of the L*P*P of a dense G_i product.
#include "common.hpp"

#include <algorithm>

namespace sg {
namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsBudget = 60 * 1024;

template <int LMAX>
__global__ __launch_bounds__(kThreads) void kron_matvec_kernel(
    int n, int P, int L, int T, int R, int ent_cap, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double* __restrict__ vals,
    const int32_t* __restrict__ kptr, const int32_t* __restrict__ tij,
    const double* __restrict__ tval, const double* __restrict__ X, double* Y,
    double alpha, double beta, const double* C) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* W = reinterpret_cast<double*>(smem_raw);            // R*L*P
    double* sv = W + (size_t)R * L * P;                           // ent_cap*L
    double* stv = sv + (size_t)ent_cap * L;                       // T
    int32_t* sc = reinterpret_cast<int32_t*>(stv + T);            // ent_cap
    int32_t* stij = sc + ent_cap;                                 // T
    int32_t* skp = stij + T;                                      // P+1
    int32_t* srp = skp + P + 1;                                   // R+1

    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * R;
    const int rows = min(R, n - row0);
    if (rows <= 0) return;
    const int e0 = rowptr[row0];
    const int e1 = rowptr[row0 + rows];
    const int ne = e1 - e0;

    for (int q = tid; q <= rows; q += kThreads) srp[q] = rowptr[row0 + q] - e0;
    for (int q = tid; q < ne; q += kThreads) sc[q] = col[e0 + q];
    for (int q = tid; q < ne * L; q += kThreads) sv[q] = vals[(size_t)e0 * L + q];
    for (int q = tid; q < T; q += kThreads) {
        stij[q] = tij[q];
        stv[q] = tval[q];
    }
    for (int q = tid; q <= P; q += kThreads) skp[q] = kptr[q];
    __syncthreads();

    // phase 1
    const int pairs = rows * P;
    for (int pq = tid; pq < pairs; pq += kThreads) {
        const int r = pq / P;
        const int j = pq - r * P;
        double acc[LMAX];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) acc[i] = 0.0;
        const int q1 = srp[r + 1];
        for (int q = srp[r]; q < q1; ++q) {
            const double x = X[(size_t)sc[q] * P + j];
            const double* v = sv + (size_t)q * L;
#pragma unroll
            for (int i = 0; i < LMAX; ++i)
                if (i < L) acc[i] = fma(v[i], x, acc[i]);
        }
        double* w = W + (size_t)r * L * P + j;
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i < L) w[(size_t)i * P] = acc[i];
    }
    __syncthreads();

    // phase 2
    for (int pq = tid; pq < pairs; pq += kThreads) {
        const int r = pq / P;
        const int k = pq - r * P;
        const double* w = W + (size_t)r * L * P;
        double acc = 0.0;
        const int t1 = skp[k + 1];
        for (int t = skp[k]; t < t1; ++t) acc = fma(stv[t], w[stij[t]], acc);
        const size_t o = (size_t)(row0 + r) * P + k;
        double outv = alpha * acc;
        if (beta != 0.0) outv = fma(beta, C[o], outv);
        Y[o] = outv;
    }
}

}  // namespace

void kron_matvec(const KronCsr& A, int L, const TriplesDev& tr, const double* X, double* Y,
                 double alpha, double beta, const double* C, hipStream_t s) {
    const int P = tr.P, T = tr.T;
    if (A.n == 0) return;
    // rows per tile: as many as fit the thread count and the LDS budget
    auto lds_for = [&](int R) {
        size_t ent = (size_t)R * A.max_row;
        return (size_t)R * L * P * 8 + ent * L * 8 + (size_t)T * 8 + ent * 4 + (size_t)T * 4 +
               (size_t)(P + 1) * 4 + (size_t)(R + 1) * 4 + 64;
    };
    int R = std::max(1, kThreads / P);
    while (R > 1 && lds_for(R) > kLdsBudget) --R;
    size_t lds = lds_for(R);
    if (lds > kLdsBudget)
        SG_THROW(SG_ERR_UNSUPPORTED, "matvec tile needs %zu bytes of LDS (P=%d L=%d T=%d)", lds, P,
                 L, T);
    int ent_cap = R * A.max_row;
    int blocks = (A.n + R - 1) / R;
#define SG_LAUNCH_MV(LM)                                                                      \
    kron_matvec_kernel<LM><<<blocks, kThreads, lds, s>>>(A.n, P, L, T, R, ent_cap, A.rowptr,  \
                                                         A.col, A.vals, tr.kptr.p, tr.tij.p,  \
                                                         tr.tval.p, X, Y, alpha, beta, C)
    if (L <= 8)
        SG_LAUNCH_MV(8);
    else if (L <= 16)
        SG_LAUNCH_MV(16);
    else if (L <= 32)
        SG_LAUNCH_MV(32);
    else
        SG_THROW(SG_ERR_UNSUPPORTED, "L_in=%d exceeds 32 in the matvec", L);
#undef SG_LAUNCH_MV
    HIP_LAUNCH_OK();
}

}  // namespace sg

using namespace sg;

extern "C" int sg_matvec(const sg_op* op, const double* X, double* Y, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && X && Y, "null argument");
        SG_REQUIRE(X != Y, "X and Y must not alias");
        check_device(op->device);
        kron_matvec(op->csr(), op->L, op->tr, X, Y, 1.0, 0.0, nullptr, as_stream(stream));
        return SG_OK;
    });
}
