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
#include "sgtable.hpp"

#include <algorithm>
#include <utility>

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

// ---------------------------------------------------------------------------
// Wide kernel (L > 32 input terms, e.g. the degree-2p coefficient fields of
// a Newton Jacobian, or P > 64 output modes).  One wave per row: the row's K_i values
// (entries x L) and its neighbours' X rows are staged in the wave's own LDS
// slice (zero-padded to EMAX entries), then every lane walks its chunk of
// the k-sorted triple table,
//     acc += m_ijk * sum_e K_i[a, b_e] X[b_e, j],
// flushing acc into a slot at the end of each run of equal k; lane k then
// sums the slots of k in order.  Work per row is T*EMAX FMAs, spread evenly
// over the 64 lanes whatever the number of triples per k.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

template <int EMAX>
__global__ __launch_bounds__(256) void kron_matvec_wide_kernel(
    int n, int P, int L, int nslot, int wpg, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double* __restrict__ vals,
    const int32_t* __restrict__ lane_ptr, const uint32_t* __restrict__ sched,
    const double* __restrict__ sval, const int32_t* __restrict__ slot_ptr,
    const double* __restrict__ X, double* Y, double alpha, double beta, const double* C) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t per_wave = (size_t)EMAX * (L + P) + nslot;
    double* Kv = reinterpret_cast<double*>(smem_raw) + wave * per_wave;   // [EMAX][L]
    double* Xv = Kv + (size_t)EMAX * L;                                    // [EMAX][P]
    double* part = Xv + (size_t)EMAX * P;                                  // [nslot]
    const int t0 = lane_ptr[lane], t1 = lane_ptr[lane + 1];
    for (int row = blockIdx.x * wpg + wave; row < n; row += gridDim.x * wpg) {
        const int e0 = rowptr[row];
        const int ne = rowptr[row + 1] - e0;
        for (int q = lane; q < EMAX * L; q += 64)
            Kv[q] = (q < ne * L) ? vals[(size_t)e0 * L + q] : 0.0;
        for (int q = lane; q < EMAX * P; q += 64) {
            const int e = q / P, j = q - (q / P) * P;
            Xv[q] = (e < ne) ? X[(size_t)col[e0 + e] * P + j] : 0.0;
        }
        wave_lds_sync();
        double acc = 0.0;
        for (int t = t0; t < t1; ++t) {
            const uint32_t w = sched[t];
            const int i = (int)(w & 0xffffu), j = (int)((w >> 16) & 0x7fu);
            double x = 0.0;
#pragma unroll
            for (int e = 0; e < EMAX; ++e) x = fma(Kv[e * L + i], Xv[e * P + j], x);
            acc = fma(sval[t], x, acc);
            if (w >> 31) {
                part[(w >> 23) & 0xffu] = acc;
                acc = 0.0;
            }
        }
        wave_lds_sync();
        for (int k = lane; k < P; k += 64) {
            double y = 0.0;
            for (int q = slot_ptr[k]; q < slot_ptr[k + 1]; ++q) y += part[q];
            const size_t o = (size_t)row * P + k;
            double outv = alpha * y;
            if (beta != 0.0) outv = fma(beta, C[o], outv);
            Y[o] = outv;
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Specialised kernel for a fixed basis (M, PIN, PO), ELL width S and IG lanes
// per row.  Each lane keeps its row's K_i values for its share of the input
// terms in registers (read once, coalesced, from the wave-tiled ELL copy),
// loops over the output columns j with X[b, j] gathered from the S
// neighbours, forms w_i = sum_s K_i[a, b_s] X[b_s, j] and scatters
// m_ijk w_i into register-resident y_k with the triple coefficients as
// immediates.  The IG partial sums of a row are combined by lane shuffles.
// Value of the partner lane (lane ^ 1): DPP quad permutation [1,0,3,2].
__device__ __forceinline__ double swap_lane_pair(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <class H, int T>
__device__ __forceinline__ void triple_step(const double* w, double* y) {
    constexpr int k = H::t.k[T];
    constexpr int ii = H::t.ii[T];
    constexpr double m = H::t.m[T];
    y[k] = fma(m, w[ii], y[k]);
}

template <class H, int T0, int... Is>
__device__ __forceinline__ void triple_range(std::integer_sequence<int, Is...>, const double* w,
                                             double* y) {
    (triple_step<H, T0 + Is>(w, y), ...);
}

template <class H, int T>
__device__ __forceinline__ void pair_step(double sel, const double* w, double* y) {
    constexpr int k = H::t.k[T];
    constexpr int ii = H::t.ii[T];
    constexpr double m0 = H::t.m0[T], d = H::t.m1[T] - H::t.m0[T];
    // sel is 0 for the first lane of a row and 1 for the second
    y[k] = fma(fma(sel, d, m0), w[ii], y[k]);
}

template <class H, int T0, int... Is>
__device__ __forceinline__ void pair_range(std::integer_sequence<int, Is...>, double sel,
                                           const double* w, double* y) {
    (pair_step<H, T0 + Is>(sel, w, y), ...);
}

template <int M, int PIN, int PO, int IG, int G, int J>
__device__ __forceinline__ void contract_j(const double* w, double* y) {
    using H = tab::GroupHolder<M, PIN, PO, IG, G>;
    constexpr int t0 = H::t.jptr[J], t1 = H::t.jptr[J + 1];
    triple_range<H, t0>(std::make_integer_sequence<int, t1 - t0>{}, w, y);
}

template <int M, int PIN, int PO, int S, int IG, int J>
__device__ __forceinline__ void column_step(int ig, const int* b, const double (*v)[(tab::cbinom(M + PIN, PIN) + IG - 1) / IG],
                                            const double* __restrict__ X, double* y) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int L = tab::cbinom(M + PIN, PIN);
    constexpr int LI = (L + IG - 1) / IG;
    double x[S];
#pragma unroll
    for (int q = 0; q < S; ++q) x[q] = X[(size_t)b[q] * P + J];
    double w[LI];
#pragma unroll
    for (int ii = 0; ii < LI; ++ii) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) a = fma(v[q][ii], x[q], a);
        w[ii] = a;
    }
    if constexpr (IG == 1) {
        contract_j<M, PIN, PO, IG, 0, J>(w, y);
    } else {
        static_assert(IG == 2, "IG must be 1 or 2");
        using H = tab::PairHolder<M, PIN, PO>;
        constexpr int t0 = H::t.jptr[J], t1 = H::t.jptr[J + 1];
        pair_range<H, t0>(std::make_integer_sequence<int, t1 - t0>{}, (double)ig, w, y);
    }
}

template <int M, int PIN, int PO, int S, int IG, int... Js>
__device__ __forceinline__ void all_columns(std::integer_sequence<int, Js...>, int ig, const int* b,
                                            const double (*v)[(tab::cbinom(M + PIN, PIN) + IG - 1) / IG],
                                            const double* __restrict__ X, double* y) {
    (column_step<M, PIN, PO, S, IG, Js>(ig, b, v, X, y), ...);
}

template <int M, int PIN, int PO, int S, int IG>
__global__ __launch_bounds__(kThreads) void kron_matvec_spec_kernel(
    int n, const int32_t* __restrict__ ecol, const double* __restrict__ evals,
    const double* __restrict__ X, double* Y, double alpha, double beta, const double* C) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int L = tab::cbinom(M + PIN, PIN);
    constexpr int LI = (L + IG - 1) / IG;
    constexpr int RW = 64 / IG;
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int r = lane / IG;
    const int ig = lane - r * IG;
    if (tile * RW >= n) return;               // whole wave past the last row
    const int row = tile * RW + r;
    int b[S];
    double v[S][LI];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        b[q] = ecol[((size_t)tile * S + q) * RW + r];
#pragma unroll
        for (int ii = 0; ii < LI; ++ii) {
            const int i = ig * LI + ii;
            v[q][ii] = (i < L) ? evals[(((size_t)tile * S + q) * L + i) * RW + r] : 0.0;
        }
    }
    double y[P];
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = 0.0;
    all_columns<M, PIN, PO, S, IG>(std::make_integer_sequence<int, P>{}, ig, b, v, X, y);
    if constexpr (IG == 2) {
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] += swap_lane_pair(y[k]);
    }
    if (row >= n || ig != 0) return;     // the first lane of a row writes it
    double* yr = Y + (size_t)row * P;
    // C may alias Y: the whole row of C is read before any of Y is written,
    // so the loads are not serialised behind the stores
    if (beta != 0.0) {
        double c[P];
#pragma unroll
        for (int k = 0; k < P; ++k) c[k] = C[(size_t)row * P + k];
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] = fma(beta, c[k], alpha * y[k]);
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] *= alpha;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) yr[k] = y[k];
}

// ---------------------------------------------------------------------------
// Split kernel for a fixed basis (M, PIN, PO) and at most S entries per row.
// A work-group of 2 KT waves covers KT tiles of 64 consecutive rows (KT = 1,
// 2 or 4, chosen per operator by timing).  Even waves take the first half of
// the input terms, odd waves the second half, each for the 64 rows of its
// tile with one row per lane.  With
// the input terms split between waves instead of between lanes, every triple
// a wave executes belongs to it and the coefficients stay immediates.  The
// neighbour rows of the block -- a few runs of consecutive rows, found at
// setup -- are staged in LDS JC columns at a time (double-buffered through
// registers) and shared by the two halves; the second half's partial sums
// reach the first through LDS.
namespace split {
constexpr int kRuns = 4, JC = 7, RB = 64;
constexpr int kRunWords = 2 * kRuns + 1;
constexpr int kTileChoices[] = {1, 2, 4};    // tiles of RB rows per work-group
constexpr int kNumTileChoices = 3;
// work-group shape for KT tiles: one wave per (tile, half), two staged rows
// per thread
template <int KT>
struct Shape {
    static constexpr int kBlockRows = KT * RB;
    static constexpr int kThreads = 2 * 64 * KT;
    static constexpr int kSlots = 2 * kThreads;
};

// Block b is dispatched to XCD b % 8; return the block id that makes XCD x
// take the x-th contiguous share of [0, nb) in order.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = (nb + 7) / 8, full = (nb % 8 == 0) ? 8 : nb % 8;
    const int x = b & 7, q = b >> 3;
    return x < full ? x * per + q : full * per + (x - full) * (per - 1) + q;
}

template <class H, int T>
__device__ __forceinline__ void tstep(const double* w, double* y) {
    constexpr int k = H::t.k[T];
    constexpr int ii = H::t.ii[T];
    constexpr double m = H::t.m[T];
    y[k] = fma(m, w[ii], y[k]);
}

template <class H, int T0, int... Is>
__device__ __forceinline__ void trange(std::integer_sequence<int, Is...>, const double* w, double* y) {
    (tstep<H, T0 + Is>(w, y), ...);
}

template <int S, int J, int J0>
__device__ __forceinline__ void xload(const int* slot, const double* xs, double* x) {
#pragma unroll
    for (int q = 0; q < S; ++q) x[q] = xs[slot[q] * JC + (J - J0)];
}

template <int M, int PIN, int PO, int S, int G, int LI, int J>
__device__ __forceinline__ void contract(const double (*v)[8], const double* x, double* y) {
    double w[LI];
#pragma unroll
    for (int ii = 0; ii < LI; ++ii) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) a = fma(v[q][ii], x[q], a);
        w[ii] = a;
    }
    using H = tab::GroupHolder<M, PIN, PO, 2, G>;
    constexpr int t0 = H::t.jptr[J], t1 = H::t.jptr[J + 1];
    trange<H, t0>(std::make_integer_sequence<int, t1 - t0>{}, w, y);
}

// Column J of a chunk: fetch column J+1's neighbour values, then contract J.
template <int M, int PIN, int PO, int S, int G, int LI, int J, int J0, int JE>
__device__ __forceinline__ void column(const int* slot, const double (*v)[8], const double* xs,
                                       double (*xb)[S], double* y) {
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (J + 1 < JE) xload<S, J + 1, J0>(slot, xs, xb[(J + 1 - J0) & 1]);
    contract<M, PIN, PO, S, G, LI, J>(v, xb[(J - J0) & 1], y);
}

template <int M, int PIN, int PO, int S, int G, int LI, int J0, int... Js>
__device__ __forceinline__ void columns(std::integer_sequence<int, Js...>, const int* slot,
                                        const double (*v)[8], const double* xs, double* y) {
    constexpr int JE = J0 + (int)sizeof...(Js);
    double xb[2][S];
    xload<S, J0, J0>(slot, xs, xb[0]);
    (column<M, PIN, PO, S, G, LI, J0 + Js, J0, JE>(slot, v, xs, xb, y), ...);
}

template <int P, int C>
constexpr int chunk_width() {
    return (P - C * JC) < JC ? (P - C * JC) : JC;
}

// Global -> registers for chunk C: each thread owns staging slots tid and
// tid + 256 (rows clamped to a valid row, so the loads never branch).
template <int P, int C>
__device__ __forceinline__ void stage_load(const double* __restrict__ X, const int* srow,
                                           double (*st)[JC]) {
    constexpr int W = chunk_width<P, C>();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double* p = X + (size_t)srow[m] * P + C * JC;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) st[m][jj] = p[jj];
    }
}

template <int P, int C, int KT>
__device__ __forceinline__ void stage_store(double* buf, int tid, const double (*st)[JC]) {
    constexpr int W = chunk_width<P, C>();
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int jj = 0; jj < W; ++jj)
            buf[(tid + Shape<KT>::kThreads * m) * JC + jj] = st[m][jj];
}

template <int M, int PIN, int PO, int S, int G, int LI, int P, int NCH, int KT, int C>
__device__ __forceinline__ void chunk(const int* slot, const double (*v)[8], double* lds,
                                      double (*st)[JC], const double* __restrict__ X,
                                      const int* srow, int tid, double* y) {
    constexpr int NS = Shape<KT>::kSlots;
    if constexpr (C + 1 < NCH) stage_load<P, C + 1>(X, srow, st);
    columns<M, PIN, PO, S, G, LI, C * JC>(std::make_integer_sequence<int, chunk_width<P, C>()>{},
                                          slot, v, lds + (C & 1) * NS * JC, y);
    if constexpr (C + 1 < NCH) stage_store<P, C + 1, KT>(lds + ((C + 1) & 1) * NS * JC, tid, st);
    __syncthreads();
}

template <int M, int PIN, int PO, int S, int G, int LI, int P, int NCH, int KT, int... Cs>
__device__ __forceinline__ void chunks(std::integer_sequence<int, Cs...>, const int* slot,
                                       const double (*v)[8], double* lds, double (*st)[JC],
                                       const double* __restrict__ X, const int* srow, int tid,
                                       double* y) {
    (chunk<M, PIN, PO, S, G, LI, P, NCH, KT, Cs>(slot, v, lds, st, X, srow, tid, y), ...);
}

// Matrix-free values (lattice meshes).  Row a sits at lattice node (i, j)
// with six elements around it; with L(ci,cj) = (v(ci,cj), v(ci+1,cj),
// v(ci+1,cj+1)) and U(ci,cj) = (v(ci,cj), v(ci+1,cj+1), v(ci,cj+1)) they are,
// with the local index of a: L(i,j):0, U(i,j):0, L(i-1,j):1, L(i-1,j-1):2,
// U(i-1,j-1):1, U(i,j-1):2.  K_i[a, b] = sum over the elements holding a and
// b of c_i(T) |T| grad phi_a . grad phi_b, with c_i(T) = c0(T) g(T)^alpha_i /
// alpha_i! regenerated from the element's fields (Eq. inputlogn).  Stencil
// directions in column order: S = 5: south, west, centre, east, north; S = 7
// adds south-west first and north-east last.  Entries of eliminated
// (boundary) neighbours are zero.
struct MfArgs {
    int N = 0;                          // lattice cells per side
    const int16_t* sdir = nullptr;      // [tiles][S][64] staging index per direction
    const double* ef = nullptr;         // [n_tri][M+1]
    const double* ek6 = nullptr;        // [n_tri][6] or null (uniform lattice)
    double ekL[6], ekU[6];
};

// contribution (direction, local pair) of the element in role r; pair indices
// 0..5 = (00, 11, 22, 01, 12, 02); direction ids: 0 S, 1 W, 2 C, 3 E, 4 N,
// 5 SW, 6 NE
struct MfContrib {
    int dir, pair;
};
constexpr MfContrib kMfRole[6][3] = {
    {{2, 0}, {3, 3}, {6, 5}},   // L(i,j):     a = 0: centre 00, east 01, north-east 02
    {{2, 0}, {4, 5}, {6, 3}},   // U(i,j):     a = 0: centre 00, north 02, north-east 01
    {{2, 1}, {1, 3}, {4, 4}},   // L(i-1,j):   a = 1: centre 11, west 10, north 12
    {{2, 2}, {0, 4}, {5, 5}},   // L(i-1,j-1): a = 2: centre 22, south 21, south-west 20
    {{2, 1}, {1, 4}, {5, 3}},   // U(i-1,j-1): a = 1: centre 11, west 12, south-west 10
    {{2, 2}, {3, 4}, {0, 5}},   // U(i,j-1):   a = 2: centre 22, east 21, south 20
};

template <int S>
constexpr int mf_slot(int dir) {
    // slot of a direction in column order, -1 when the pattern has none
    if constexpr (S == 5) {
        return dir <= 4 ? dir : -1;
    } else {
        return dir == 5 ? 0 : dir == 6 ? 6 : dir + 1;
    }
}

template <int M, int PO, int I>
__device__ __forceinline__ double monomial(const double* f) {
    // c0 prod_m g_m^alpha_m / alpha_m! for input term I
    constexpr const auto& b = tab::BasisHolder<M, PO>::b;
    double r = f[0];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int am = b.a[I][m];
        if (am >= 1) r *= f[1 + m];
        if (am >= 2) r *= 0.5 * f[1 + m];
    }
    return r;
}

// The contributions of one element (role r, fields f, masked weights w) to
// the values of input terms I0 + IIs.
template <int M, int PO, int S, int I0, int... IIs>
__device__ __forceinline__ void mf_terms(std::integer_sequence<int, IIs...>, int r, const double* f,
                                         const double* w, double (*v)[8]) {
    (
        [&] {
            const double cb = monomial<M, PO, I0 + IIs>(f);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int sl = mf_slot<S>(kMfRole[r][c].dir);
                if (sl >= 0) v[sl][IIs] = fma(cb, w[c], v[sl][IIs]);
            }
        }(),
        ...);
}

template <int M, int PIN, int PO, int S, int G>
__device__ __forceinline__ void mf_values(int row, int n, const MfArgs& mf, double (*v)[8]) {
    constexpr int L = tab::cbinom(M + PIN, PIN);
    constexpr int LH = (L + 1) / 2;
    constexpr int LI = G == 0 ? LH : L - LH;
    static_assert(PIN <= 2, "the matrix-free values cover input orders <= 2");
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
        for (int ii = 0; ii < LI; ++ii) v[q][ii] = 0.0;
    if (row >= n) return;
    const int N = mf.N, Nm = N - 1;
    const int i = row % Nm + 1, j = row / Nm + 1;
    const double mask[7] = {j > 1 ? 1.0 : 0.0, i > 1 ? 1.0 : 0.0, 1.0, i < Nm ? 1.0 : 0.0,
                            j < Nm ? 1.0 : 0.0, (i > 1 && j > 1) ? 1.0 : 0.0,
                            (i < Nm && j < Nm) ? 1.0 : 0.0};
    const int cell[6] = {j * N + i, j * N + i, j * N + i - 1, (j - 1) * N + i - 1,
                         (j - 1) * N + i - 1, (j - 1) * N + i};
    constexpr int lu[6] = {0, 1, 0, 0, 1, 1};
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int64_t e = 2 * (int64_t)cell[r] + lu[r];
        double f[M + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m) f[m] = mf.ef[e * (M + 1) + m];
        double w[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int pr = kMfRole[r][c].pair;
            w[c] = mf.ek6 ? mf.ek6[e * 6 + pr] : (lu[r] ? mf.ekU[pr] : mf.ekL[pr]);
            w[c] *= mask[kMfRole[r][c].dir];
        }
        mf_terms<M, PO, S, G * LH>(std::make_integer_sequence<int, LI>{}, r, f, w, v);
    }
}

// One half of the input terms over the whole row: G = 0 takes i < ceil(L/2).
template <int M, int PIN, int PO, int S, int G, int KT, bool MF>
__device__ __forceinline__ void half(int tile, int r, const int* slot,
                                     const double* __restrict__ svals, const MfArgs& mf, int n,
                                     double* lds, double (*st)[JC], const double* __restrict__ X,
                                     const int* srow, int tid, double* y) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int L = tab::cbinom(M + PIN, PIN);
    constexpr int LH = (L + 1) / 2;
    constexpr int LI = G == 0 ? LH : L - LH;
    constexpr int NCH = (P + JC - 1) / JC;
    static_assert(LH <= 8, "half of the input terms must fit 8 registers per entry");
    double v[S][8];
    if constexpr (MF) {
        mf_values<M, PIN, PO, S, G>(tile * RB + r, n, mf, v);
    } else {
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int ii = 0; ii < LI; ++ii)
                v[q][ii] = svals[(((size_t)tile * S + q) * L + G * LH + ii) * RB + r];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = 0.0;
    __syncthreads();   // chunk 0 staged
    chunks<M, PIN, PO, S, G, LI, P, NCH, KT>(std::make_integer_sequence<int, NCH>{}, slot, v, lds,
                                             st, X, srow, tid, y);
}

template <int M, int PIN, int PO, int S, int KT, bool MF = false>
__global__ __launch_bounds__(Shape<KT>::kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void kron_matvec_split_kernel(int n, int ntiles, const int32_t* __restrict__ runs,
                              const int16_t* __restrict__ sslot, const double* __restrict__ svals,
                              const double* __restrict__ X, double* Y, double alpha, double beta,
                              const double* C, MfArgs mf) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int kThreads = Shape<KT>::kThreads, kSlots = Shape<KT>::kSlots;
    static_assert(KT * P * RB <= 2 * kSlots * JC, "partial sums must fit the staging area");
    __shared__ double lds[2 * kSlots * JC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Work-groups are dealt to the 8 XCDs in turn; renumber them so that each
    // XCD walks one contiguous range of row blocks, and the neighbour rows a
    // block stages were mostly fetched into the same L2 by its predecessors.
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int32_t* rw = runs + (size_t)blk * kRunWords;
    int rrow[kRuns], rslot[kRuns];
#pragma unroll
    for (int q = 0; q < kRuns; ++q) {
        rrow[q] = rw[q];
        rslot[q] = rw[kRuns + q];
    }
    const int nslot = rw[2 * kRuns];
    int srow[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int sl = tid + kThreads * m;
        int row = rrow[0] + (sl - rslot[0]);
#pragma unroll
        for (int q = 1; q < kRuns; ++q) row = (sl >= rslot[q]) ? rrow[q] + (sl - rslot[q]) : row;
        srow[m] = (sl < nslot) ? row : rrow[0];
    }
    double st[2][JC];
    stage_load<P, 0>(X, srow, st);
    stage_store<P, 0, KT>(lds, tid, st);

    const int g = wave & 1, rb = wave >> 1;
    const int tile = blk * KT + rb;
    const bool live = tile < ntiles;
    const int tt = live ? tile : 0;
    int slot[S];
    const int16_t* sl16 = MF ? mf.sdir : sslot;
#pragma unroll
    for (int q = 0; q < S; ++q) slot[q] = sl16[((size_t)tt * S + q) * RB + lane];
    double y[P];
    const int nrows = live ? n : 0;      // a dead wave's tile forms no values
    if (g == 0)
        half<M, PIN, PO, S, 0, KT, MF>(tt, lane, slot, svals, mf, nrows, lds, st, X, srow, tid, y);
    else
        half<M, PIN, PO, S, 1, KT, MF>(tt, lane, slot, svals, mf, nrows, lds, st, X, srow, tid, y);
    // the staging area is free after the last chunk's barrier
    if (g == 1) {
#pragma unroll
        for (int k = 0; k < P; ++k) lds[(rb * P + k) * RB + lane] = y[k];
    }
    __syncthreads();
    const int row = tile * RB + lane;
    if (g == 1 || !live || row >= n) return;
    double* yr = Y + (size_t)row * P;
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = alpha * (y[k] + lds[(rb * P + k) * RB + lane]);
    // C may alias Y: the whole row of C is read before any of Y is written,
    // so the loads are not serialised behind the stores
    if (beta != 0.0) {
        double c[P];
#pragma unroll
        for (int k = 0; k < P; ++k) c[k] = C[(size_t)row * P + k];
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] = fma(beta, c[k], y[k]);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) yr[k] = y[k];
}
}  // namespace split

// ---------------------------------------------------------------------------
// Grouped kernel for wide fixed bases (many input terms and output modes,
// e.g. M = 6, p = 3: L_in = 28, P = 84, on the 7-point pattern of a jittered
// mesh).  One work-group takes one tile of 64 rows with IGN x KGN waves.
// Wave (ig, kg) holds, one row per lane, the K values of the input terms
// [ig*LI, ig*LI + LI) of its row's entries and accumulates the output modes
// [kg*KL, kg*KL + KL), so both the values and the accumulators fit the
// registers of two waves per SIMD; the coefficients m_ijk of each wave's
// share stay immediates.  The tile's neighbour rows (a few runs of
// consecutive rows, as for the split kernel) are staged in LDS JC columns at
// a time, double-buffered through registers, and shared by all waves; JC is
// odd, so the 8-byte reads of consecutive rows hit distinct banks.  The
// waves of one input-term group add their partial sums through LDS at the
// end, in a fixed order.
namespace grp {
constexpr int RB = 64, JC = 13, kSlots = 256;
using split::kRuns;
using split::kRunWords;

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) const uint32_t glb_u32;

template <int P, int C>
constexpr int width() {
    return (P - C * JC) < JC ? (P - C * JC) : JC;
}

constexpr int kBufDoubles = kSlots * JC;          // one staged chunk: [slot][JC]
constexpr int kDmaBlocks = kBufDoubles * 2 / 64;  // 64 dwords per wave-wide DMA
static_assert(kBufDoubles * 2 % 64 == 0, "a chunk must be whole DMA blocks");

// LDS: two chunk buffers, each its own array.  A DMA into one array does
// not make the compiler wait for it before reads of the other (it keeps the
// two apart; slices of one array it could not), so chunk C + 1 streams in
// while chunk C is read.  After the last chunk the buffers take the partial
// sums of the input-term groups, one group at a time, output group kg in
// buffer kg.  The dynamic LDS holds the source row of each staging slot and
// the staging offset of each entry of the tile's rows.
template <int S>
constexpr size_t kTableDoubles = (kSlots + S * RB + 1) / 2;

template <int P, int S>
constexpr size_t lds_doubles(int IGN, int KGN) {
    return kTableDoubles<S>;
}

// Stage chunk C of the tile's neighbour rows into buf by LDS DMA: dword d of
// the chunk is half (d & 1) of X[row(slot)][C*JC + jj], slot*JC + jj = d / 2.
// Wave w issues the 64-dword blocks w, w + NW, ...; no registers hold the
// values, and the loads stay in flight until the wave's vmcnt wait.
template <int P, int C, int NW>
__device__ __forceinline__ void stage_dma(const double* __restrict__ X, const int* srows,
                                          double* buf, int wave, int lane) {
    constexpr int W = width<P, C>();
    for (int blk = wave; blk < kDmaBlocks; blk += NW) {
        const int d = blk * 64 + lane;
        const int e = d >> 1;
        const int slot = e / JC, jj = e - slot * JC;
        const int col = C * JC + (jj < W ? jj : 0);     // positions past the chunk read column 0
        const uint32_t* src =
            reinterpret_cast<const uint32_t*>(X + (size_t)srows[slot] * P + col) + (d & 1);
        __builtin_amdgcn_global_load_lds((glb_u32*)src, (lds_u32*)((char*)buf + blk * 256), 4, 0,
                                         0);
    }
}

__device__ __forceinline__ void dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// slot: staging offsets in doubles (staging slot * JC).  The reads are
// volatile: every wave group reads the same addresses, and merging those
// reads across the groups' branches would hoist them and keep many columns'
// values live at once.
template <int S, int JJ>
__device__ __forceinline__ void xload(const int* slot, const double* xs, double* x) {
    typedef const volatile __attribute__((address_space(3))) double lds_cvd;
    lds_cvd* vx = (lds_cvd*)xs;
#pragma unroll
    for (int q = 0; q < S; ++q) x[q] = vx[slot[q] + JJ];
}

// The triples of one column (sorted by input term) form each
// w = sum_q K_i[a, b_q] X[b_q, j] just before the triples that use it, so only
// one w is live.
template <class H, int J>
constexpr bool has_triples() {
    return H::t.jptr[J + 1] > H::t.jptr[J];
}

template <class H, int S, int LI, int T0, int T>
__device__ __forceinline__ void wstep(const double (*v)[LI], const double* x, double& w,
                                      double* y) {
    constexpr int ii = H::t.ii[T];
    if constexpr (T == T0 || H::t.ii[T > T0 ? T - 1 : T0] != ii) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) a = fma(v[q][ii], x[q], a);
        w = a;
    }
    constexpr int k = H::t.k[T];
    constexpr double m = H::t.m[T];
    y[k] = fma(m, w, y[k]);
}

template <class H, int S, int LI, int T0, int... Is>
__device__ __forceinline__ void wrange(std::integer_sequence<int, Is...>, const double (*v)[LI],
                                       const double* x, double* y) {
    double w = 0.0;
    (wstep<H, S, LI, T0, T0 + Is>(v, x, w, y), ...);
}

// Column J0 + JJ for the wave group of H: load the neighbour values, then
// walk the column's triples.
template <class H, int S, int LI, int J0, int JJ>
__device__ __forceinline__ void column(const int* slot, const double (*v)[LI], const double* xs,
                                       double* y) {
    if constexpr (has_triples<H, J0 + JJ>()) {
        constexpr int t0 = H::t.jptr[J0 + JJ], t1 = H::t.jptr[J0 + JJ + 1];
        // columns are not interleaved by the scheduler: that would keep more
        // products live than the registers hold
        __builtin_amdgcn_sched_barrier(0);
        double x[S];
        xload<S, JJ>(slot, xs, x);
        wrange<H, S, LI, t0>(std::make_integer_sequence<int, t1 - t0>{}, v, x, y);
    }
}

template <class H, int S, int LI, int J0, int... JJs>
__device__ __forceinline__ void columns(std::integer_sequence<int, JJs...>, const int* slot,
                                        const double (*v)[LI], const double* xs, double* y) {
    (column<H, S, LI, J0, JJs>(slot, v, xs, y), ...);
}

// The columns of chunk C for the wave's group (one branch per group and
// chunk).  The staging offsets of the rows' entries are read from LDS at the
// start of the chunk, so they are not kept in registers across chunks.
template <int M, int PIN, int PO, int S, int IGN, int KGN, int LI, int C, int... Gs>
__device__ __forceinline__ void chunk_groups(std::integer_sequence<int, Gs...>, int wave, int lane,
                                             const int* soff, const double (*v)[LI],
                                             const double* xs, double* y) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int W = width<P, C>();
    int slot[S];
#pragma unroll
    for (int q = 0; q < S; ++q) slot[q] = soff[q * RB + lane];
    ((wave == Gs ? (columns<tab::WaveGroupHolder<M, PIN, PO, IGN, KGN, Gs>, S, LI, C * JC>(
                        std::make_integer_sequence<int, W>{}, slot, v, xs, y),
                    0)
                 : 0),
     ...);
}

template <int M, int PIN, int PO, int S, int IGN, int KGN, int LI, int NCH, int... Cs>
__device__ __forceinline__ void chunks(std::integer_sequence<int, Cs...>, int wave, int lane,
                                       const int* srows, const int* soff, const double (*v)[LI],
                                       double* buf0, double* buf1, const double* __restrict__ X,
                                       double* y) {
    constexpr int P = tab::cbinom(M + PO, PO);
    (([&] {
         // chunk Cs + 1 streams into the other buffer (last read in chunk Cs - 1,
         // before the barrier that ended it) while chunk Cs is computed
         if constexpr (Cs + 1 < NCH)
             stage_dma<P, Cs + 1, IGN * KGN>(X, srows, (Cs + 1) & 1 ? buf1 : buf0, wave, lane);
         chunk_groups<M, PIN, PO, S, IGN, KGN, LI, Cs>(
             std::make_integer_sequence<int, IGN * KGN>{}, wave, lane, soff, v,
             Cs & 1 ? buf1 : buf0, y);
         dma_wait();
         __syncthreads();
     }()),
     ...);
}

template <int M, int PIN, int PO, int S, int IGN, int KGN>
__global__ __launch_bounds__(64 * IGN * KGN) __attribute__((amdgpu_waves_per_eu(2, 2)))
void kron_matvec_group_kernel(int n, int ntiles, const int32_t* __restrict__ runs,
                              const int16_t* __restrict__ sslot, const double* __restrict__ svals,
                              const double* __restrict__ X, double* Y, double alpha, double beta,
                              const double* C) {
    constexpr int P = tab::cbinom(M + PO, PO);
    constexpr int L = tab::cbinom(M + PIN, PIN);
    constexpr int LI = (L + IGN - 1) / IGN, KL = (P + KGN - 1) / KGN;
    constexpr int NCH = (P + JC - 1) / JC;
    constexpr int kThreads = 64 * IGN * KGN;
    static_assert(kThreads >= kSlots && kThreads >= S * RB, "threads for the LDS tables");
    static_assert(KGN <= 2 && KL * RB <= kBufDoubles, "partial sums of a group fit one buffer");
    __shared__ __align__(16) double buf0[kBufDoubles];
    __shared__ __align__(16) double buf1[kBufDoubles];
    extern __shared__ __align__(16) double glds[];
    int* srows = reinterpret_cast<int*>(glds);
    int* soff = srows + kSlots;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ig = wave % IGN, kg = wave / IGN;
    const int tile = split::xcd_block(blockIdx.x, gridDim.x);
    // source row of every staging slot (slots past the runs read a valid row),
    // and the staging offset (in doubles) of every entry of the tile's rows
    if (tid < kSlots) {
        const int32_t* rw = runs + (size_t)tile * kRunWords;
        int r = rw[0] + (tid - rw[kRuns]);
#pragma unroll
        for (int q = 1; q < kRuns; ++q) r = (tid >= rw[kRuns + q]) ? rw[q] + (tid - rw[kRuns + q]) : r;
        srows[tid] = tid < rw[2 * kRuns] ? r : rw[0];
    }
    if (tid < S * RB) soff[tid] = (int)sslot[(size_t)tile * S * RB + tid] * JC;
    double v[S][LI];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
        for (int ii = 0; ii < LI; ++ii) {
            const int i = ig * LI + ii;
            v[q][ii] = i < L ? svals[(((size_t)tile * S + q) * L + i) * RB + lane] : 0.0;
        }
    __syncthreads();                                  // tables ready
    stage_dma<P, 0, IGN * KGN>(X, srows, buf0, wave, lane);
    double y[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) y[k] = 0.0;
    dma_wait();
    __syncthreads();                                  // chunk 0 staged
    chunks<M, PIN, PO, S, IGN, KGN, LI, NCH>(std::make_integer_sequence<int, NCH>{}, wave, lane,
                                             srows, soff, v, buf0, buf1, X, y);
    // partial sums of input-term groups 1.. through LDS (the staging buffers
    // are free), added to group 0's in group order
    double* red = kg == 0 ? buf0 : buf1;
    for (int g2 = 1; g2 < IGN; ++g2) {
        if (ig == g2) {
#pragma unroll
            for (int k = 0; k < KL; ++k) red[(size_t)k * RB + lane] = y[k];
        }
        __syncthreads();
        if (ig == 0) {
#pragma unroll
            for (int k = 0; k < KL; ++k) y[k] += red[(size_t)k * RB + lane];
        }
        __syncthreads();
    }
    if (ig > 0) return;
    const int row = tile * RB + lane;
    if (row >= n) return;
    const int k0 = kg * KL;
    double* yr = Y + (size_t)row * P + k0;
    if (beta != 0.0) {
        // C may alias Y: this wave's part of the row of C is read before any
        // of Y is written
        double c[KL];
#pragma unroll
        for (int k = 0; k < KL; ++k) c[k] = (k0 + k < P) ? C[(size_t)row * P + k0 + k] : 0.0;
#pragma unroll
        for (int k = 0; k < KL; ++k) y[k] = fma(beta, c[k], alpha * y[k]);
    } else {
#pragma unroll
        for (int k = 0; k < KL; ++k) y[k] *= alpha;
    }
#pragma unroll
    for (int k = 0; k < KL; ++k)
        if (k0 + k < P) yr[k] = y[k];
}
}  // namespace grp

// ---------------------------------------------------------------------------
// Row-tiled kernel for wide input bases (L > 32 input terms, P <= 48 output
// modes, at most 7 entries per row), e.g. the degree-2p coefficient fields of
// a Newton Jacobian.  One work-group per tile of 64 rows, one lane per row:
//   - the tile's neighbour rows are staged once in LDS by output column
//     ([j][slot]), so lane a reads X[b_e, j] at its own slot of column j;
//   - its K values pass through LDS in chunks of 8 input terms
//     ([entry][term][lane], two buffers, the next chunk's loads in flight
//     under the current chunk's products);
//   - in each chunk, each of the 16 waves owns up to 3 output modes k
//     (assigned on the host, chunk by chunk, to balance the chunk's triple
//     counts, since the waves meet at a barrier after every chunk), takes
//     their running sums from LDS into registers, walks the list of the
//     chunk's triples (i, j, k) of its modes, forming
//         y_k += m_ijk sum_e K_i[a, b_e] X[b_e, j],
//     and puts the sums back.  The list is the same for every lane: it is
//     read in batches of 8 entries (scalar loads, one wait per batch), and
//     each LDS access is lane-contiguous (K, sums) or a row's own slot (X).
// Every lane does T * 7 FMAs per row with 14 LDS reads each; the one-wave-
// per-row kernel does the same work with lane-dependent (conflicting) LDS
// addresses.
namespace rowt {
constexpr int RB = 64, S = 7, NW = 16, KS = 3, IC = 8, TB = 8;
constexpr int kSlots = 256;                       // staged neighbour rows of one tile
constexpr int kXs = kSlots + 1;                   // doubles per staged column (odd: spreads banks)
constexpr int kThreads = 64 * NW;
constexpr int kChunk = S * IC * RB;               // doubles of one K chunk
constexpr int kPer = (kChunk + kThreads - 1) / kThreads;
constexpr int kYs = RB + 1;                       // doubles per mode row of the sums
static_assert(RB == split::RB, "the tile staging is the split kernel's one-tile staging");
inline size_t lds_bytes(int P) {
    return ((size_t)P * kXs + 2 * (size_t)kChunk + (size_t)P * kYs) * sizeof(double);
}

__global__ __launch_bounds__(kThreads) void kron_matvec_rowtile_kernel(
    int n, int P, int L, int nch, const int32_t* __restrict__ runs,
    const int16_t* __restrict__ sslot, const double* __restrict__ svals,
    const int32_t* __restrict__ lptr, const uint32_t* __restrict__ lij,
    const double* __restrict__ lm, const int32_t* __restrict__ wk, const double* __restrict__ X,
    double* Y, double alpha, double beta, const double* C) {
    using split::kRuns;
    extern __shared__ __align__(16) double rl[];
    double* Xs = rl;                                  // [P][kXs]
    double* Kb = rl + (size_t)P * kXs;                // [2][S][IC][RB]
    double* Ys = Kb + 2 * (size_t)kChunk;             // [P][kYs] running sums
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tile = blockIdx.x;
    const int32_t* rw = runs + (size_t)tile * split::kRunWords;
    int rrow[kRuns], rsl[kRuns];
#pragma unroll
    for (int u = 0; u < kRuns; ++u) {
        rrow[u] = rw[u];
        rsl[u] = rw[kRuns + u];
    }
    const int nslot = rw[2 * kRuns];
    // neighbour rows, column by column (a run of slots is a run of rows, so
    // consecutive threads read consecutive words of X)
    for (int q = tid; q < nslot * P; q += kThreads) {
        const int sl = q / P, j = q - sl * P;
        int r = rrow[0] + (sl - rsl[0]);
#pragma unroll
        for (int u = 1; u < kRuns; ++u) r = (sl >= rsl[u]) ? rrow[u] + (sl - rsl[u]) : r;
        Xs[(size_t)j * kXs + sl] = X[(size_t)r * P + j];
    }
    for (int q = tid; q < P * kYs; q += kThreads) Ys[q] = 0.0;
    int xo[S];
#pragma unroll
    for (int e = 0; e < S; ++e) xo[e] = sslot[((size_t)tile * S + e) * RB + lane];
    const double* kt = svals + (size_t)tile * S * L * RB;   // [S][L][RB]
    const uint64_t* lmb = reinterpret_cast<const uint64_t*>(lm);
    static_assert(TB == 8, "the batch barrier below names 8 entries");
    double v[kPer];
    auto kload = [&](int c) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = tid + u * kThreads;
            const int qq = q < kChunk ? q : 0;
            const int e = qq / (IC * RB), il = (qq / RB) % IC, ln = qq % RB;
            const int i = c * IC + il;
            v[u] = (q < kChunk && i < L) ? kt[((size_t)e * L + i) * RB + ln] : 0.0;
        }
    };
    auto kstore = [&](double* buf) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = tid + u * kThreads;
            if (q < kChunk) buf[q] = v[u];
        }
    };
    kload(0);
    kstore(Kb);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const double* cur = Kb + (size_t)(c & 1) * kChunk + lane;
        const bool more = c + 1 < nch;
        if (more) kload(c + 1);
        // this chunk's modes of the wave (each mode has one owner per chunk;
        // the barrier at the end of a chunk orders the hand-over)
        int ks[KS];
        double y[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            ks[s] = wk[((size_t)c * NW + wave) * KS + s];
            y[s] = ks[s] >= 0 ? Ys[(size_t)ks[s] * kYs + lane] : 0.0;
        }
        const int t1 = lptr[c * NW + wave + 1];
        for (int tb = lptr[c * NW + wave]; tb < t1; tb += TB) {
            // a batch of list entries (the list array is padded by TB
            // entries, so the batch never reads past it)
            uint32_t wv[TB];
            uint64_t mb[TB];
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                wv[u] = lij[tb + u];
                mb[u] = lmb[tb + u];
            }
            // all of the batch's scalar loads are taken here, with one wait
            // (the compiler would otherwise move each load to its use)
            asm volatile("" ::"s"(wv[0]), "s"(wv[1]), "s"(wv[2]), "s"(wv[3]), "s"(wv[4]),
                         "s"(wv[5]), "s"(wv[6]), "s"(wv[7]), "s"(mb[0]), "s"(mb[1]), "s"(mb[2]),
                         "s"(mb[3]), "s"(mb[4]), "s"(mb[5]), "s"(mb[6]), "s"(mb[7]));
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                if (tb + u >= t1) break;
                const double* kb = cur + (wv[u] & 0xffu) * RB;
                const double* xb = Xs + (size_t)((wv[u] >> 8) & 0xffu) * kXs;
                double x = 0.0;
#pragma unroll
                for (int e = 0; e < S; ++e) x = fma(kb[e * IC * RB], xb[xo[e]], x);
                const double m = __longlong_as_double((long long)mb[u]);
                const uint32_t sl = wv[u] >> 16;
#pragma unroll
                for (int s = 0; s < KS; ++s)
                    if (sl == (uint32_t)s) y[s] = fma(m, x, y[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (ks[s] >= 0) Ys[(size_t)ks[s] * kYs + lane] = y[s];
        if (more) kstore(Kb + (size_t)((c + 1) & 1) * kChunk);
        __syncthreads();
    }
    // the tile's outputs, row-major (contiguous stores)
    const int row0 = tile * RB;
    const int rows = min(RB, n - row0);
    for (int q = tid; q < rows * P; q += kThreads) {
        const int r = q / P, k = q - r * P;
        const size_t o = (size_t)row0 * P + q;
        double outv = alpha * Ys[(size_t)k * kYs + r];
        if (beta != 0.0) outv = fma(beta, C[o], outv);   // C may alias Y: read before the write
        Y[o] = outv;
    }
}
}  // namespace rowt

// ELL copy: entry id of every (tile, slot, lane) position, -1 for padding.
__global__ void ell_fill_kernel(int64_t npos, int L, int S, int RW, const int64_t* __restrict__ ent,
                                const double* __restrict__ vals, double* __restrict__ evals) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npos * L) return;
    // idx enumerates ((tile*S + s)*L + i)*RW + r
    const int64_t r = idx % RW;
    const int64_t i = (idx / RW) % L;
    const int64_t ts = idx / ((int64_t)RW * L);
    const int64_t e = ent[ts * RW + r];
    evals[idx] = e >= 0 ? vals[e * L + i] : 0.0;
}

struct Spec {
    int M, PIN, PO, S, IG;
};
constexpr Spec kSpecs[] = {{2, 2, 2, 5, 1}, {2, 2, 2, 7, 1}, {4, 2, 3, 5, 2}, {4, 2, 3, 7, 2}};

template <int Id>
void launch_spec(const KronCsr& A, const double* X, double* Y, double alpha, double beta,
                 const double* C, hipStream_t s) {
    constexpr Spec sp = kSpecs[Id];
    constexpr int RW = 64 / sp.IG;
    const int tiles = (A.n + RW - 1) / RW;
    const int blocks = (tiles + kThreads / 64 - 1) / (kThreads / 64);
    kron_matvec_spec_kernel<sp.M, sp.PIN, sp.PO, sp.S, sp.IG>
        <<<blocks, kThreads, 0, s>>>(A.n, A.ecol, A.evals, X, Y, alpha, beta, C);
}

struct SplitSpec {
    int M, PIN, PO, S;
};
constexpr SplitSpec kSplits[] = {{2, 2, 2, 5}, {2, 2, 2, 7}, {4, 2, 3, 5}};

template <int Id, int KT>
void launch_split_kt(const KronCsr& A, const double* X, double* Y, double alpha, double beta,
                     const double* C, hipStream_t s) {
    constexpr SplitSpec sp = kSplits[Id];
    using Sh = split::Shape<KT>;
    const int tiles = (A.n + split::RB - 1) / split::RB;
    const int blocks = (A.n + Sh::kBlockRows - 1) / Sh::kBlockRows;
    split::MfArgs mf;
    if (A.mf) {
        mf.N = A.mf_N;
        mf.sdir = A.sdir;
        mf.ef = A.ef;
        mf.ek6 = A.ek6;
        for (int q = 0; q < 6; ++q) {
            mf.ekL[q] = A.ekL[q];
            mf.ekU[q] = A.ekU[q];
        }
        split::kron_matvec_split_kernel<sp.M, sp.PIN, sp.PO, sp.S, KT, true>
            <<<blocks, Sh::kThreads, 0, s>>>(A.n, tiles, A.sruns, A.sslot, A.svals, X, Y, alpha,
                                             beta, C, mf);
    } else {
        split::kron_matvec_split_kernel<sp.M, sp.PIN, sp.PO, sp.S, KT, false>
            <<<blocks, Sh::kThreads, 0, s>>>(A.n, tiles, A.sruns, A.sslot, A.svals, X, Y, alpha,
                                             beta, C, mf);
    }
}

template <int Id>
void launch_split(const KronCsr& A, const double* X, double* Y, double alpha, double beta,
                  const double* C, hipStream_t s) {
    switch (A.split_kt) {
        case 1: launch_split_kt<Id, 1>(A, X, Y, alpha, beta, C, s); break;
        case 2: launch_split_kt<Id, 2>(A, X, Y, alpha, beta, C, s); break;
        case 4: launch_split_kt<Id, 4>(A, X, Y, alpha, beta, C, s); break;
        default: SG_THROW(SG_ERR_INVALID_ARG, "bad tiles per work-group %d", A.split_kt);
    }
}

struct GroupSpec {
    int M, PIN, PO, S, IGN, KGN;
};
constexpr GroupSpec kGroups[] = {{6, 2, 3, 7, 4, 2}};

template <int Id>
void launch_group(const KronCsr& A, const double* X, double* Y, double alpha, double beta,
                  const double* C, hipStream_t s) {
    constexpr GroupSpec g = kGroups[Id];
    constexpr int P = tab::cbinom(g.M + g.PO, g.PO);
    const int tiles = (A.n + grp::RB - 1) / grp::RB;
    const size_t lds = grp::lds_doubles<P, g.S>(g.IGN, g.KGN) * sizeof(double);
    grp::kron_matvec_group_kernel<g.M, g.PIN, g.PO, g.S, g.IGN, g.KGN>
        <<<tiles, 64 * g.IGN * g.KGN, lds, s>>>(A.n, tiles, A.sruns, A.sslot, A.svals, X, Y, alpha,
                                                beta, C);
}

// Neighbour rows of one block of rows as at most kRuns runs of consecutive
// rows (the smallest gaps merged first), laid out one after the other in the
// staging area.  False when they need more than `slots` staged rows.
bool block_runs(std::vector<int32_t>& cols, int slots, int32_t* words) {
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    std::vector<int32_t> start, end;   // [start, end)
    for (size_t u = 0; u < cols.size();) {
        size_t w = u + 1;
        while (w < cols.size() && cols[w] == cols[w - 1] + 1) ++w;
        start.push_back(cols[u]);
        end.push_back(cols[w - 1] + 1);
        u = w;
    }
    while ((int)start.size() > split::kRuns) {
        size_t best = 1;
        for (size_t q = 2; q < start.size(); ++q)
            if (start[q] - end[q - 1] < start[best] - end[best - 1]) best = q;
        end[best - 1] = end[best];
        start.erase(start.begin() + best);
        end.erase(end.begin() + best);
    }
    int base = 0;
    for (int q = 0; q < split::kRuns; ++q) {
        const bool used = q < (int)start.size();
        words[q] = used ? start[q] : start[0];
        words[split::kRuns + q] = used ? base : (1 << 30);
        if (used) base += end[q] - start[q];
    }
    words[2 * split::kRuns] = base;
    return base <= slots;
}

// Staging index of column c in a block whose runs are `w`.
int16_t staged_index(const int32_t* w, int32_t c) {
    int q = split::kRuns - 1;
    while (w[split::kRuns + q] == (1 << 30) || c < w[q]) --q;
    return (int16_t)(w[split::kRuns + q] + (c - w[q]));
}

// Per block of KT tiles: the runs, and per (tile, entry, lane) the staging
// index of the entry's column.  False when a block does not fit.
bool split_staging(const sg_op* op, int S, int KT, std::vector<int32_t>& runs,
                   std::vector<int16_t>& slot) {
    const int RB = split::RB, n = op->n;
    const int rows = KT * RB, slots = 2 * 2 * 64 * KT;
    const int tiles = (n + RB - 1) / RB;
    const int blocks = (n + rows - 1) / rows;
    runs.assign((size_t)blocks * split::kRunWords, 0);
    slot.assign((size_t)tiles * S * RB, 0);
    std::vector<int32_t> cols;
    for (int blk = 0; blk < blocks; ++blk) {
        const int a0 = blk * rows, a1 = std::min(n, a0 + rows);
        cols.assign(op->h_col.begin() + op->h_rowptr[a0], op->h_col.begin() + op->h_rowptr[a1]);
        for (int a = a0; a < a1; ++a) cols.push_back(a);   // padding entries read the own row
        int32_t* w = runs.data() + (size_t)blk * split::kRunWords;
        if (!block_runs(cols, slots, w)) return false;
        auto staged = [&](int32_t c) { return staged_index(w, c); };
        for (int a = a0; a < a1; ++a) {
            const int t = a / RB, r = a % RB;
            int q = 0;
            for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e, ++q)
                slot[((size_t)t * S + q) * RB + r] = staged(op->h_col[e]);
            for (; q < S; ++q) slot[((size_t)t * S + q) * RB + r] = staged(a);
        }
    }
    return true;
}

// Matrix-free staging for KT tiles per work-group: per (tile, direction,
// lane) the staging index of the row's neighbour in that stencil direction
// (its own row where the neighbour is eliminated).  False when the tile
// count does not fit or the pattern is not exactly the lattice stencil
// (every direction present, or the neighbour eliminated).
bool mf_staging(const sg_op* op, int S, int KT, std::vector<int16_t>& sdir) {
    std::vector<int32_t> runs;
    std::vector<int16_t> slot;
    if (!split_staging(op, S, KT, runs, slot)) return false;
    const int RB = split::RB, n = op->n, Nm = op->lattice_N - 1;
    const int rows = KT * RB, tiles = (n + RB - 1) / RB;
    sdir.assign((size_t)tiles * S * RB, 0);
    for (int a = 0; a < n; ++a) {
        const int32_t* w = runs.data() + (size_t)(a / rows) * split::kRunWords;
        const int i = a % Nm + 1, j = a / Nm + 1;
        int nb[7], cnt = 0;
        std::vector<int32_t> want;
        auto add = [&](bool present, int32_t b) {
            nb[cnt++] = present ? b : a;
            if (present) want.push_back(b);
        };
        if (S == 7) add(i > 1 && j > 1, a - Nm - 1);
        add(j > 1, a - Nm);
        add(i > 1, a - 1);
        add(true, a);
        add(i < Nm, a + 1);
        add(j < Nm, a + Nm);
        if (S == 7) add(i < Nm && j < Nm, a + Nm + 1);
        std::vector<int32_t> have(op->h_col.begin() + op->h_rowptr[a],
                                  op->h_col.begin() + op->h_rowptr[a + 1]);
        std::sort(want.begin(), want.end());
        if (have != want) return false;
        const int t = a / RB, r = a % RB;
        for (int q = 0; q < S; ++q) sdir[((size_t)t * S + q) * RB + r] = staged_index(w, nb[q]);
    }
    return true;
}

// Staged copy for the split kernel: the L values per (tile, entry, lane),
// and the staging of every tile count that fits (two tiles per group when
// that fits, the default until sg_matvec_autotune or sg_matvec_select).
bool build_split(sg_op* op, hipStream_t s) {
    const sg_basis& b = op->basis;
    int id = -1;
    for (int q = 0; q < (int)(sizeof(kSplits) / sizeof(kSplits[0])); ++q) {
        const SplitSpec& sp = kSplits[q];
        if (sp.M == b.M && sp.PIN == b.p_in && sp.PO == b.p && op->max_row <= sp.S) {
            id = q;
            break;
        }
    }
    if (id < 0 || op->n == 0) return false;
    const int S = kSplits[id].S, RB = split::RB;
    const int n = op->n;
    const int tiles = (n + RB - 1) / RB;
    bool any = false;
    std::vector<int32_t> runs;
    std::vector<int16_t> slot;
    for (int v = 0; v < split::kNumTileChoices; ++v) {
        op->split_fits[v] = split_staging(op, S, split::kTileChoices[v], runs, slot);
        if (!op->split_fits[v]) continue;
        op->sruns[v].upload(runs, s);
        op->sslot[v].upload(slot, s);
        any = true;
    }
    if (!any) return false;
    std::vector<int64_t> ent((size_t)tiles * S * RB, -1);
    for (int a = 0; a < n; ++a) {
        const int t = a / RB, r = a % RB;
        int q = 0;
        for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e, ++q)
            ent[((size_t)t * S + q) * RB + r] = e;
    }
    DevBuf<int64_t> d_ent;
    d_ent.upload(ent, s);
    const int64_t npos = (int64_t)tiles * S * RB;
    op->svals.alloc((size_t)npos * op->L);
    ell_fill_kernel<<<(unsigned)((npos * op->L + 255) / 256), 256, 0, s>>>(npos, op->L, S, RB, d_ent.p,
                                                                           op->vals.p, op->svals.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(s));
    op->split = id;
    op->split_var = op->split_fits[1] ? 1 : (op->split_fits[0] ? 0 : 2);
    return true;
}

// Staged copy for the grouped kernel: one tile of 64 rows per work-group, the
// values per (tile, entry, lane) and the staging of each tile's neighbour rows.
bool build_group(sg_op* op, hipStream_t s) {
    const sg_basis& b = op->basis;
    int id = -1;
    for (int q = 0; q < (int)(sizeof(kGroups) / sizeof(kGroups[0])); ++q) {
        const GroupSpec& g = kGroups[q];
        if (g.M == b.M && g.PIN == b.p_in && g.PO == b.p && op->max_row <= g.S) {
            id = q;
            break;
        }
    }
    if (id < 0 || op->n == 0) return false;
    const int S = kGroups[id].S, RB = grp::RB;
    static_assert(grp::RB == split::RB && grp::kSlots == 2 * 2 * split::RB,
                  "the grouped kernel reuses the one-tile staging of the split kernel");
    std::vector<int32_t> runs;
    std::vector<int16_t> slot;
    if (!split_staging(op, S, 1, runs, slot)) return false;
    int lds_max = 0;
    HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device));
    const GroupSpec g = kGroups[id];
    const int P = op->P;
    const size_t need = (2 * (size_t)grp::kBufDoubles + (grp::kSlots + (size_t)S * RB + 1) / 2) * 8;
    if (need > (size_t)lds_max) return false;
    op->sruns[0].upload(runs, s);
    op->sslot[0].upload(slot, s);
    const int n = op->n, tiles = (n + RB - 1) / RB;
    std::vector<int64_t> ent((size_t)tiles * S * RB, -1);
    for (int a = 0; a < n; ++a) {
        const int t = a / RB, r = a % RB;
        int q = 0;
        for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e, ++q)
            ent[((size_t)t * S + q) * RB + r] = e;
    }
    DevBuf<int64_t> d_ent;
    d_ent.upload(ent, s);
    const int64_t npos = (int64_t)tiles * S * RB;
    op->svals.alloc((size_t)npos * op->L);
    ell_fill_kernel<<<(unsigned)((npos * op->L + 255) / 256), 256, 0, s>>>(npos, op->L, S, RB, d_ent.p,
                                                                           op->vals.p, op->svals.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(s));
    op->group = id;
    op->split_var = 0;
    return true;
}

}  // namespace

void build_ell(sg_op* op, hipStream_t s) {
    op->spec = -1;
    op->split = -1;
    op->group = -1;
    if (build_split(op, s)) return;
    if (build_group(op, s)) return;
    const sg_basis& b = op->basis;
    int id = -1;
    for (int q = 0; q < (int)(sizeof(kSpecs) / sizeof(kSpecs[0])); ++q) {
        const Spec& sp = kSpecs[q];
        if (sp.M == b.M && sp.PIN == b.p_in && sp.PO == b.p && op->max_row <= sp.S) {
            id = q;
            break;
        }
    }
    if (id < 0) {
        build_row_tiled(op, s);
        return;
    }
    const Spec sp = kSpecs[id];
    const int RW = 64 / sp.IG;
    const int n = op->n;
    const int tiles = (n + RW - 1) / RW;
    std::vector<int32_t> ecol((size_t)tiles * sp.S * RW, 0);
    std::vector<int64_t> ent((size_t)tiles * sp.S * RW, -1);
    for (int a = 0; a < n; ++a) {
        const int t = a / RW, r = a % RW;
        int q = 0;
        for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e, ++q) {
            ecol[((size_t)t * sp.S + q) * RW + r] = op->h_col[e];
            ent[((size_t)t * sp.S + q) * RW + r] = e;
        }
        for (; q < sp.S; ++q) ecol[((size_t)t * sp.S + q) * RW + r] = a;   // padding: own row, value 0
    }
    op->ecol.upload(ecol, s);
    DevBuf<int64_t> d_ent;
    d_ent.upload(ent, s);
    const int64_t npos = (int64_t)tiles * sp.S * RW;
    op->evals.alloc((size_t)npos * op->L);
    ell_fill_kernel<<<(unsigned)((npos * op->L + 255) / 256), 256, 0, s>>>(npos, op->L, sp.S, RW,
                                                                           d_ent.p, op->vals.p,
                                                                           op->evals.p);
    HIP_LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(s));
    op->spec = id;
    op->ell_S = sp.S;
    op->ell_RW = RW;
}

bool build_row_tiled(sg_op* op, hipStream_t s) {
    using namespace rowt;
    const sg_basis& b = op->basis;
    const int P = op->P, L = op->L, n = op->n;
    op->rt_built = op->rt_on = false;
    if (n == 0 || L <= 32 || P > NW * KS || op->max_row > S || b.tk.empty()) return false;
    if (op->split >= 0 || op->group >= 0) return false;
    int lds_max = 0;
    HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device));
    if (lds_bytes(P) > (size_t)lds_max) return false;
    std::vector<int32_t> runs;
    std::vector<int16_t> slot;
    if (!split_staging(op, S, 1, runs, slot)) return false;
    // per chunk of input terms: the chunk's output modes to (wave, slot),
    // largest triple count in the chunk first, each to the least loaded wave
    // with a free slot; then per (chunk, wave) the wave's triples ordered by
    // (i, j, k), entry = (i - chunk start) | j << 8 | slot << 16
    const int nch = (L + IC - 1) / IC;
    std::vector<int> tord(b.tk.size());
    for (size_t t = 0; t < tord.size(); ++t) tord[t] = (int)t;
    std::sort(tord.begin(), tord.end(), [&](int x, int y) {
        if (b.ti[x] != b.ti[y]) return b.ti[x] < b.ti[y];
        if (b.tj[x] != b.tj[y]) return b.tj[x] < b.tj[y];
        return b.tk[x] < b.tk[y];
    });
    std::vector<int32_t> wk((size_t)nch * NW * KS, -1);
    std::vector<int32_t> lptr;
    std::vector<uint32_t> lij;
    std::vector<double> lm;
    for (int c = 0; c < nch; ++c) {
        std::vector<int> cnt(P, 0), kw(P, -1), ksl(P, -1);
        for (int t : tord)
            if (b.ti[t] / IC == c) ++cnt[b.tk[t]];
        std::vector<int> order(P);
        for (int k = 0; k < P; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cnt[x] > cnt[y]; });
        std::vector<int> load(NW, 0), used(NW, 0);
        for (int k : order) {
            if (cnt[k] == 0) continue;
            int best = -1;
            for (int w = 0; w < NW; ++w)
                if (used[w] < KS && (best < 0 || load[w] < load[best])) best = w;
            if (best < 0) return false;
            kw[k] = best;
            ksl[k] = used[best];
            wk[((size_t)c * NW + best) * KS + used[best]++] = k;
            load[best] += cnt[k];
        }
        for (int w = 0; w < NW; ++w) {
            lptr.push_back((int32_t)lij.size());
            for (int t : tord) {
                if (b.ti[t] / IC != c || kw[b.tk[t]] != w) continue;
                lij.push_back((uint32_t)(b.ti[t] % IC) | ((uint32_t)b.tj[t] << 8) |
                              ((uint32_t)ksl[b.tk[t]] << 16));
                lm.push_back(b.tv[t]);
            }
        }
    }
    lptr.push_back((int32_t)lij.size());
    lij.resize(lij.size() + TB, 0u);                  // batches read up to TB entries ahead
    lm.resize(lm.size() + TB, 0.0);
    const int tiles = (n + RB - 1) / RB;
    std::vector<int64_t> ent((size_t)tiles * S * RB, -1);
    for (int a = 0; a < n; ++a) {
        const int t = a / RB, r = a % RB;
        int q = 0;
        for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e, ++q)
            ent[((size_t)t * S + q) * RB + r] = e;
    }
    op->sruns[0].upload(runs, s);
    op->sslot[0].upload(slot, s);
    op->rt_lptr.upload(lptr, s);
    op->rt_lij.upload(lij, s);
    op->rt_lm.upload(lm, s);
    op->rt_wk.upload(wk, s);
    op->rt_ent.upload(ent, s);
    op->svals.alloc((size_t)tiles * S * RB * L);
    op->rt_nch = nch;
    op->rt_built = op->rt_on = true;
    refresh_row_tiled(op, s);
    HIP_OK(hipStreamSynchronize(s));   // the host vectors are freed on return
    return true;
}

void refresh_row_tiled(sg_op* op, hipStream_t s) {
    if (!op->rt_built) return;
    const int64_t npos = (int64_t)((op->n + rowt::RB - 1) / rowt::RB) * rowt::S * rowt::RB;
    ell_fill_kernel<<<(unsigned)((npos * op->L + 255) / 256), 256, 0, s>>>(
        npos, op->L, rowt::S, rowt::RB, op->rt_ent.p, op->vals.p, op->svals.p);
    HIP_LAUNCH_OK();
}

void kron_matvec(const KronCsr& A, int L, const TriplesDev& tr, const double* X, double* Y,
                 double alpha, double beta, const double* C, hipStream_t s) {
    const int P = tr.P, T = tr.T;
    if (A.n == 0) return;
    if (A.group >= 0) {
        switch (A.group) {
            case 0: launch_group<0>(A, X, Y, alpha, beta, C, s); break;
            default: SG_THROW(SG_ERR_INVALID_ARG, "bad grouped matvec variant %d", A.group);
        }
        HIP_LAUNCH_OK();
        return;
    }
    if (A.split >= 0) {
        switch (A.split) {
            case 0: launch_split<0>(A, X, Y, alpha, beta, C, s); break;
            case 1: launch_split<1>(A, X, Y, alpha, beta, C, s); break;
            case 2: launch_split<2>(A, X, Y, alpha, beta, C, s); break;
            default: SG_THROW(SG_ERR_INVALID_ARG, "bad matvec split variant %d", A.split);
        }
        HIP_LAUNCH_OK();
        return;
    }
    if (A.spec >= 0) {
        switch (A.spec) {
            case 0: launch_spec<0>(A, X, Y, alpha, beta, C, s); break;
            case 1: launch_spec<1>(A, X, Y, alpha, beta, C, s); break;
            case 2: launch_spec<2>(A, X, Y, alpha, beta, C, s); break;
            case 3: launch_spec<3>(A, X, Y, alpha, beta, C, s); break;
            default: SG_THROW(SG_ERR_INVALID_ARG, "bad matvec specialisation %d", A.spec);
        }
        HIP_LAUNCH_OK();
        return;
    }
    if (A.rowt) {
        const int tiles = (A.n + rowt::RB - 1) / rowt::RB;
        rowt::kron_matvec_rowtile_kernel<<<tiles, rowt::kThreads, rowt::lds_bytes(P), s>>>(
            A.n, P, L, A.rt_nch, A.sruns, A.sslot, A.svals, A.rt_lptr, A.rt_lij, A.rt_lm, A.rt_wk,
            X, Y, alpha, beta, C);
        HIP_LAUNCH_OK();
        return;
    }
    // many input terms, or outputs too wide for the tiled kernel's LDS budget:
    // one wave per row with the balanced triple schedule
    if (L > 32 || P > 64) {
        SG_REQUIRE(tr.nslot > 0, "wide matvec schedule missing");
        int emax = A.max_row <= 7 ? 7 : A.max_row <= 10 ? 10 : A.max_row <= 16 ? 16 : 0;
        if (!emax) SG_THROW(SG_ERR_UNSUPPORTED, "wide matvec: %d entries in a row exceed 16", A.max_row);
        const size_t per_wave = ((size_t)emax * (L + P) + tr.nslot) * 8;
        const size_t cap = 64 * 1024;
        int wpg = (int)std::min<size_t>(4, cap / per_wave);
        if (wpg < 1)
            SG_THROW(SG_ERR_UNSUPPORTED, "wide matvec row needs %zu bytes of LDS (L=%d P=%d)", per_wave,
                     L, P);
        const size_t lds = per_wave * wpg;
        const int blocks = (int)std::min<int64_t>((A.n + wpg - 1) / wpg, 8192);
#define SG_LAUNCH_WIDE(EM)                                                                   \
    kron_matvec_wide_kernel<EM><<<blocks, 64 * wpg, lds, s>>>(                               \
        A.n, P, L, tr.nslot, wpg, A.rowptr, A.col, A.vals, tr.lane_ptr.p, tr.sched.p, tr.tval.p, \
        tr.slot_ptr.p, X, Y, alpha, beta, C)
        if (emax == 7)
            SG_LAUNCH_WIDE(7);
        else if (emax == 10)
            SG_LAUNCH_WIDE(10);
        else
            SG_LAUNCH_WIDE(16);
#undef SG_LAUNCH_WIDE
        HIP_LAUNCH_OK();
        return;
    }
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

namespace sg {
void linop_apply(const LinOp& A, const double* X, double* Y, double alpha, double beta,
                 const double* C, hipStream_t s) {
    kron_matvec(A.kron->csr(), A.kron->L, A.kron->tr, X, Y, alpha, beta, C, s);
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

extern "C" int sg_matvec_matrix_free(sg_op* op, int enable, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op != nullptr, "op is NULL");
        check_device(op->device);
        if (!enable) {
            if (op->mf_on) graph_cache_purge(op);
            op->mf_on = false;
            return SG_OK;
        }
        if (op->split < 0 || op->lattice_N <= 0 || op->basis.p_in > 2 || !op->mf_ef.p)
            SG_THROW(SG_ERR_UNSUPPORTED,
                     "the matrix-free apply needs a lattice mesh and a basis with the staged "
                     "matvec (input order <= 2)");
        hipStream_t s = as_stream(stream);
        const int S = kSplits[op->split].S;
        bool any = false;
        for (int v = 0; v < split::kNumTileChoices; ++v) {
            if (op->mf_fits[v] || !op->split_fits[v]) continue;
            std::vector<int16_t> sdir;
            op->mf_fits[v] = mf_staging(op, S, split::kTileChoices[v], sdir);
            if (op->mf_fits[v]) op->mf_sdir[v].upload(sdir, s);
        }
        for (int v = 0; v < split::kNumTileChoices; ++v) any |= op->mf_fits[v];
        if (!any || !op->mf_fits[op->split_var])
            SG_THROW(SG_ERR_UNSUPPORTED, "the pattern is not the lattice stencil");
        HIP_OK(hipStreamSynchronize(s));
        if (!op->mf_on) graph_cache_purge(op);
        op->mf_on = true;
        return SG_OK;
    });
}

extern "C" int sg_matvec_row_tiled(sg_op* op, int enable) {
    return guarded([&]() -> int {
        SG_REQUIRE(op != nullptr, "op is NULL");
        check_device(op->device);
        if (enable && !op->rt_built)
            SG_THROW(SG_ERR_UNSUPPORTED, "the operator has no row-tiled matvec");
        if (op->rt_on != (enable != 0)) graph_cache_purge(op);
        op->rt_on = enable != 0;
        return SG_OK;
    });
}

extern "C" int sg_matvec_kernel(const sg_op* op, int* kind) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && kind, "null argument");
        if (op->mf_on && op->split >= 0)
            *kind = SG_MV_MATRIX_FREE;
        else if (op->rt_built && op->rt_on && op->split < 0 && op->group < 0)
            *kind = SG_MV_ROW_TILED;
        else if (op->group >= 0)
            *kind = SG_MV_GROUPED;
        else if (op->split >= 0)
            *kind = SG_MV_STAGED;
        else if (op->spec >= 0)
            *kind = SG_MV_PAIR;
        else if (op->L > 32 || op->P > 64)
            *kind = SG_MV_WIDE;
        else
            *kind = SG_MV_GENERIC;
        return SG_OK;
    });
}

extern "C" int sg_matvec_select(sg_op* op, int tiles) {
    return guarded([&]() -> int {
        SG_REQUIRE(op, "null argument");
        if (op->split < 0) SG_THROW(SG_ERR_UNSUPPORTED, "the operator has no staged matvec");
        int v = -1;
        for (int q = 0; q < split::kNumTileChoices; ++q)
            if (split::kTileChoices[q] == tiles) v = q;
        SG_REQUIRE(v >= 0, "tiles per work-group must be 1, 2 or 4 (got %d)", tiles);
        if (!op->split_fits[v] || (op->mf_on && !op->mf_fits[v]))
            SG_THROW(SG_ERR_UNSUPPORTED, "%d tiles per work-group do not fit this operator", tiles);
        if (v != op->split_var) graph_cache_purge(op);   // captured steps hold the old launch
        op->split_var = v;
        return SG_OK;
    });
}

extern "C" int sg_matvec_tiles(const sg_op* op, int* tiles) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && tiles, "null argument");
        *tiles = op->split >= 0 ? split::kTileChoices[op->split_var] : 0;
        return SG_OK;
    });
}

extern "C" int sg_matvec_autotune(sg_op* op, int reps, double* ms_out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && ms_out, "null argument");
        SG_REQUIRE(reps >= 1, "reps must be >= 1");
        check_device(op->device);
        if (op->split < 0) SG_THROW(SG_ERR_UNSUPPORTED, "the operator has no staged matvec");
        hipStream_t s = as_stream(stream);
        const size_t N = (size_t)op->n * op->P;
        DevBuf<double> X(N), Y(N);
        HIP_OK(hipMemsetAsync(X.p, 0, N * 8, s));
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        double best = -1.0;
        int best_v = op->split_var;
        for (int v = 0; v < split::kNumTileChoices; ++v) {
            ms_out[v] = -1.0;
            if (!op->split_fits[v] || (op->mf_on && !op->mf_fits[v])) continue;
            op->split_var = v;
            const KronCsr A = op->csr();
            kron_matvec(A, op->L, op->tr, X.p, Y.p, 1.0, 0.0, nullptr, s);   // warm-up
            HIP_OK(hipEventRecord(e0, s));
            for (int q = 0; q < reps; ++q) kron_matvec(A, op->L, op->tr, X.p, Y.p, 1.0, 0.0, nullptr, s);
            HIP_OK(hipEventRecord(e1, s));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            ms_out[v] = ms / reps;
            if (best < 0.0 || ms_out[v] < best) {
                best = ms_out[v];
                best_v = v;
            }
        }
        HIP_OK(hipEventDestroy(e0));
        HIP_OK(hipEventDestroy(e1));
        op->split_var = best_v;
        graph_cache_purge(op);   // captured steps hold the launch they were recorded with
        return SG_OK;
    });
}
