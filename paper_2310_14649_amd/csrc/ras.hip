// One-level restricted additive Schwarz (Eq. RASsto) with mean-based local
// solves:  Z = sum_s R_s^T D_s (R_s K_0 R_s^T)^{-1} (R_s R) G_0^{-1}.
//
// Local factorisation.  The nodes of each overlapping subdomain are ordered
// by breadth-first level sets of the local matrix graph (from a
// pseudo-peripheral node), which makes R_s K_0 R_s^T block tridiagonal:
// level l only couples to levels l-1 and l+1.  Its block LDL^T factor is
//   S_0 = A_00,  S_l = A_ll - B_l S_{l-1}^{-1} B_l^T,   B_l = A_{l,l-1},
// and the device keeps S_l^{-1} (dense, at most 64 x 64) for every level.
// A solve is a forward sweep  y_l = r_l - B_l z_{l-1},  z_l = S_l^{-1} y_l
// and a backward sweep  x_l = z_l - S_l^{-1} (B_{l+1}^T x_{l+1}).
// This is an exact solve of the mean-based local problem (the same map as a
// dense Cholesky solve, up to rounding) while storing sum_l b_l^2 entries
// instead of n_s^2.  Inverses are stored in FP64, FP32 or BF16; the low
// precisions accumulate in FP32.
//
// One work-group per (subdomain, column chunk): the P right-hand-side
// columns of a local solve are independent (G_0 is diagonal).
#include "common.hpp"

#include <algorithm>
#include <numeric>

struct sg_ras {
    int device = 0;
    int n = 0, P = 0, L = 0, n_sub = 0, overlap = 0, max_b = 0, max_local = 0, max_couple = 0,
        max_levels = 0;
    sg_prec prec = SG_FP64;
    int64_t total_local = 0, n_lev = 0, sinv_count = 0;
    std::vector<int32_t> h_nlocal, h_nlev, h_owner;
    std::vector<int32_t> h_own_ptr, h_own_nodes;   // owned nodes per subdomain
    std::vector<int32_t> h_sub_node_off, h_gnode, h_owned;   // local nodes in level order
    sg::DevBuf<int32_t> sub_node_off, sub_lev_off, lev_start, lev_size, gnode, owned, lrow_ptr,
        lcol, prev_idx, next_idx;
    sg::DevBuf<int64_t> sinv_off;
    sg::DevBuf<double> lval, sinv64, zs, afact, prev_val, next_val;
    sg::DevBuf<float> sinv32;
    sg::DevBuf<uint16_t> sinv16;
    // operator entries behind the local values (for refactorisation)
    int64_t op_nnz = 0;
    int op_L = 0;
    sg::DevBuf<int64_t> lent, prev_ent, next_ent;
    // dense path: explicit inverse rows of the owned nodes of each subdomain
    // (local columns in level order, ld = nloc padded to 64), stored in
    // tiles of 16 rows in the order the apply kernel's lanes load them
    // (n_own padded to 64 rows; offsets h_toff)
    bool dense_built = false, use_dense = false;
    int Pp = 0;                                   // P padded to 16
    std::vector<int32_t> h_ld, h_nown;
    std::vector<int64_t> h_aoff, h_toff, h_xoff;  // row-major (set-up), tiled, gathered
    sg::DevBuf<int32_t> own_pos;                  // per local node: owned index or -1
    sg::DevBuf<int32_t> ld_d, nown_d, node_sub, own_gnode;
    sg::DevBuf<int32_t> blk_sub[3], blk_row0[3];   // per variant: 64 / 32 rows per wave, fused
    sg::DevBuf<int64_t> aoff_d, toff_d, xoff_d, own_off_d;
    sg::DevBuf<double> ainv64;
    sg::DevBuf<float> ainv32;
    sg::DevBuf<uint16_t> ainv16;
    sg::DevBuf<unsigned char> xg;                 // gathered right-hand sides [s][Pp][ld]
    int nblk[3] = {0, 0, 0};
    int dense_var = 0;                            // 0: 64 rows per wave, 1: 32, 2: fused
    // Kronecker local solves (ras_set_local): the right-hand side is first
    // mixed per node by W = Gt^{-1} G_0 [P x Pw, row k col j, zero-padded] into kron_t
    sg_local_kind local_mode = SG_LOCAL_MEAN;
    sg::DevBuf<double> kron_w, kron_t;
    // the fused dense path applies the mixing to its output instead:
    // Z = N(R) Gt^{-1} with N the node operator, Gt^{-1} [P x Pp] (the
    // mixing commutes with N, and W diag(1/alpha!) = Gt^{-1}; applied in the
    // accumulator precision, FP64 for the FP64 path)
    sg::DevBuf<double> kron_post;
    bool post_ok = false;
    int post_pp = 0;                              // its column padding (P padded to 16)
    size_t post_lds = 0;
    size_t lds_max = 0;                           // LDS bytes a work-group may use
    std::vector<double> h_gt;                     // Gt, for ras_local_factor
    bool fused_ok = false;                        // fused variant fits (LDS, columns)
    size_t fused_lds = 0;                         // its LDS bytes per work-group
    double ms_sweep = -1.0, ms_dense = -1.0;      // autotuner timings
};

namespace sg {

constexpr int kRasThreads = 256;
constexpr int kMaxLevel = 64;
constexpr int kColChunk = 16;   // right-hand-side columns per work-group (one MFMA tile)
constexpr int kCouple = 8;      // max neighbours of a node in an adjacent level
constexpr int kMaxLocal = 8192;  // max nodes of one overlapping subdomain

inline size_t ras_apply_lds(sg_prec prec, int bmax, int KC, int nmax, int lmax) {
    (void)KC;
    const size_t ts = prec == SG_FP64 ? 8 : (prec == SG_FP32 ? 4 : 2);
    const int KS = prec == SG_BF16 ? 32 : 4;
    const size_t rp = ((bmax + 15) / 16) * 16, cp = ((bmax + KS - 1) / KS) * KS;
    return rp * cp * ts + cp * 16 * ts + 16 + 2 * (size_t)bmax * 16 * sizeof(double) +
           (size_t)nmax * sizeof(int32_t) + 2 * (size_t)lmax * sizeof(int32_t) + 8 +
           (size_t)lmax * sizeof(int64_t) + 16 * sizeof(double);
}

namespace {

__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Work-group barrier for LDS traffic only: waits for this wave's LDS
// operations (lgkmcnt) but not for outstanding global loads, so prefetches
// issued before the barrier stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // vmcnt=max, expcnt=max, lgkmcnt=0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <class TS> struct Load;
template <> struct Load<double> {
    using Acc = double;
    static __device__ double get(const double* p, int64_t i) { return p[i]; }
};
template <> struct Load<float> {
    using Acc = float;
    static __device__ float get(const float* p, int64_t i) { return p[i]; }
};
template <> struct Load<uint16_t> {
    using Acc = float;
    static __device__ float get(const uint16_t* p, int64_t i) { return from_bf16(p[i]); }
};

// out[q] = K_0 value of global entry ent[q] (0 where ent[q] < 0)
__global__ void gather_k0_kernel(int64_t m, int L, const int64_t* __restrict__ ent,
                                 const double* __restrict__ vals, double* __restrict__ out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) out[q] = ent[q] >= 0 ? vals[ent[q] * L] : 0.0;
}

// Block-tridiagonal factorisation, one work-group per subdomain.
__global__ __launch_bounds__(kRasThreads) void ras_factor_kernel(
    const int32_t* __restrict__ sub_node_off, const int32_t* __restrict__ sub_lev_off,
    const int32_t* __restrict__ lev_start, const int32_t* __restrict__ lev_size,
    const int64_t* __restrict__ sinv_off, const int32_t* __restrict__ lrow_ptr,
    const int32_t* __restrict__ lcol, const double* __restrict__ lval, double* __restrict__ sinv64,
    float* __restrict__ sinv32, uint16_t* __restrict__ sinv16, int prec, int* __restrict__ status) {
    extern __shared__ __align__(16) double fsm[];
    double* S = fsm;                          // b x b (current level)
    double* Sp = fsm + kMaxLevel * kMaxLevel; // previous level's inverse
    const int s = blockIdx.x, tid = threadIdx.x;
    const int node0 = sub_node_off[s];
    const int lv0 = sub_lev_off[s], lv1 = sub_lev_off[s + 1];
    for (int lv = lv0; lv < lv1; ++lv) {
        const int st = lev_start[lv], b = lev_size[lv];
        const int stp = lv > lv0 ? lev_start[lv - 1] : 0;
        const int bp = lv > lv0 ? lev_size[lv - 1] : 0;
        for (int q = tid; q < b * b; q += kRasThreads) S[q] = 0.0;
        __syncthreads();
        for (int r = tid; r < b; r += kRasThreads) {
            const int row = node0 + st + r;
            for (int q = lrow_ptr[row]; q < lrow_ptr[row + 1]; ++q) {
                const int c = lcol[q];
                if (c >= st && c < st + b) S[r * b + (c - st)] = lval[q];
            }
        }
        __syncthreads();
        if (bp > 0) {
            for (int q = tid; q < b * b; q += kRasThreads) {
                const int r = q / b, c = q - (q / b) * b;
                const int rr = node0 + st + r, rc = node0 + st + c;
                double acc = 0.0;
                for (int q1 = lrow_ptr[rr]; q1 < lrow_ptr[rr + 1]; ++q1) {
                    const int p = lcol[q1] - stp;
                    if (p < 0 || p >= bp) continue;
                    const double v1 = lval[q1];
                    for (int q2 = lrow_ptr[rc]; q2 < lrow_ptr[rc + 1]; ++q2) {
                        const int pp = lcol[q2] - stp;
                        if (pp < 0 || pp >= bp) continue;
                        acc = fma(v1 * Sp[p * bp + pp], lval[q2], acc);
                    }
                }
                S[q] -= acc;
            }
            __syncthreads();
        }
        // in-place Gauss-Jordan inversion of the SPD Schur complement
        for (int k = 0; k < b; ++k) {
            const double piv = S[k * b + k];
            if (!(piv > 0.0) || !isfinite(piv)) {
                if (tid == 0) status[0] = 1;
                return;   // uniform: every thread read the same pivot
            }
            const double ip = 1.0 / piv;
            for (int q = tid; q < b * b; q += kRasThreads) {
                const int i = q / b, j = q - (q / b) * b;
                if (i != k && j != k) S[q] = fma(-S[i * b + k] * ip, S[k * b + j], S[q]);
            }
            __syncthreads();
            for (int q = tid; q < b; q += kRasThreads) {
                if (q != k) {
                    S[k * b + q] *= ip;
                    S[q * b + k] = -S[q * b + k] * ip;
                } else {
                    S[k * b + k] = ip;
                }
            }
            __syncthreads();
        }
        const int64_t off = sinv_off[lv];
        for (int q = tid; q < b * b; q += kRasThreads) {
            const double v = S[q];
            sinv64[off + q] = v;
            if (prec == SG_FP32) sinv32[off + q] = (float)v;
            if (prec == SG_BF16) sinv16[off + q] = to_bf16((float)v);
            Sp[q] = v;
        }
        __syncthreads();
    }
}

// Per-precision matrix-core step of the level product Z_l = S_l^{-1} Y_l on a
// 16-row tile (wave w owns rows 16w..16w+15, the 16 columns of the chunk):
//   FP64: v_mfma_f64_16x16x4f64, Y in FP64;
//   FP32: v_mfma_f32_16x16x4f32, Y rounded to FP32;
//   BF16: v_mfma_f32_16x16x32_bf16, Y rounded to BF16; FP32 accumulation.
// A[i][k] sits in lane i + 16*(k / kpl) (kpl consecutive k per lane), B[k][j]
// in lane j + 16*(k / kpl); the output row of register v is row_of(lane, v)
// and its column lane % 16.
typedef double sg_d4 __attribute__((ext_vector_type(4)));
typedef float sg_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 sg_bf8 __attribute__((ext_vector_type(8)));

template <class TS> struct Mma;
template <> struct Mma<double> {
    using YT = double;
    using Acc = sg_d4;
    static constexpr int KS = 4;
    static constexpr bool ytrans = false;
    static __device__ Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ int row_of(int lane, int v) { return 4 * v + (lane >> 4); }
    static __device__ Acc step(const double* S, int cp, const double* Y, int c0, int lane, int w,
                               Acc acc) {
        const double a = S[(16 * w + (lane & 15)) * cp + c0 + (lane >> 4)];
        const double b = Y[(c0 + (lane >> 4)) * 16 + (lane & 15)];
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    static __device__ YT conv(double x) { return x; }
};
template <> struct Mma<float> {
    using YT = float;
    using Acc = sg_f4;
    static constexpr int KS = 4;
    static constexpr bool ytrans = false;
    static __device__ Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ Acc step(const float* S, int cp, const float* Y, int c0, int lane, int w,
                               Acc acc) {
        const float a = S[(16 * w + (lane & 15)) * cp + c0 + (lane >> 4)];
        const float b = Y[(c0 + (lane >> 4)) * 16 + (lane & 15)];
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    static __device__ YT conv(double x) { return (float)x; }
};
template <> struct Mma<uint16_t> {
    using YT = uint16_t;
    using Acc = sg_f4;
    static constexpr int KS = 32;
    static constexpr bool ytrans = true;      // Y stored [16][cp] so 8 k are contiguous
    static __device__ Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ Acc step(const uint16_t* S, int cp, const uint16_t* Y, int c0, int lane, int w,
                               Acc acc) {
        const uint4 a4 = *reinterpret_cast<const uint4*>(S + (16 * w + (lane & 15)) * cp + c0 + 8 * (lane >> 4));
        const uint4 b4 = *reinterpret_cast<const uint4*>(Y + (lane & 15) * cp + c0 + 8 * (lane >> 4));
        sg_bf8 a, b;
        __builtin_memcpy(&a, &a4, 16);
        __builtin_memcpy(&b, &b4, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    static __device__ YT conv(double x) { return to_bf16((float)x); }
};

// Apply: one work-group (4 waves) per (subdomain, chunk of KC <= 16
// right-hand-side columns).  The subdomain's global node ids and ownership
// flags sit in LDS for the whole sweep.  Each level: phase A forms the
// right-hand-side tile (gathered rows minus the coupling to the neighbour
// level) in the operand precision; phase B multiplies by S_l^{-1} on the
// matrix cores, one wave per 16-row tile.  Every global load a level needs is
// issued one level ahead (during the previous level's product), and the
// barriers wait for LDS traffic only, so those loads stay in flight.
// Z[owned] = beta * Z[owned] + omega * (local solution) / alpha!.
template <class TS, int KCP, int BM, bool SETUP = false>
__global__ __launch_bounds__(kRasThreads) void ras_apply_kernel(
    int P, int KC, int bmax, int nmax, int lmax, const int32_t* __restrict__ sub_node_off,
    const int32_t* __restrict__ sub_lev_off, const int32_t* __restrict__ lev_start,
    const int32_t* __restrict__ lev_size, const int64_t* __restrict__ sinv_off,
    const TS* __restrict__ sinv, const int32_t* __restrict__ gnode,
    const int32_t* __restrict__ owned, const int32_t* __restrict__ prev_idx,
    const double* __restrict__ prev_val, const int32_t* __restrict__ next_idx,
    const double* __restrict__ next_val, const double* __restrict__ afact,
    const double* __restrict__ R, double* Z, double* __restrict__ zs, double omega, double beta,
    int qbase = 0, const int32_t* __restrict__ own_pos = nullptr,
    const int32_t* __restrict__ ainv_ld = nullptr, const int64_t* __restrict__ ainv_off = nullptr,
    double* __restrict__ ainv = nullptr) {
    using MM = Mma<TS>;
    using YT = typename MM::YT;
    constexpr int KS = MM::KS;
    constexpr int RPM = ((BM + 15) / 16) * 16;
    constexpr int CPM = ((BM + KS - 1) / KS) * KS;
    constexpr int NPF = (RPM * CPM + kRasThreads - 1) / kRasThreads;
    constexpr int NQ = (CPM * 16 + kRasThreads - 1) / kRasThreads;
    constexpr int NK = CPM / KS;                  // max product steps per level
    auto rp_of = [](int b) { return ((b + 15) / 16) * 16; };
    auto cp_of = [](int b) { return ((b + KS - 1) / KS) * KS; };
    const int rpx = rp_of(bmax), cpx = cp_of(bmax);
    extern __shared__ __align__(16) unsigned char ras_smem[];
    TS* Sb = reinterpret_cast<TS*>(ras_smem);                               // rpx*cpx
    YT* Y = reinterpret_cast<YT*>(Sb + rpx * cpx);                           // cpx*16
    double* Zc = reinterpret_cast<double*>(
        (reinterpret_cast<uintptr_t>(Y + cpx * 16) + 15) & ~uintptr_t(15)); // bmax*16
    double* Zp = Zc + bmax * 16;
    int32_t* lgn = reinterpret_cast<int32_t*>(Zp + bmax * 16);               // nmax, bit 31 = owned
    int32_t* lmeta = lgn + nmax;                                             // 2*lmax: start, size
    int64_t* loff = reinterpret_cast<int64_t*>(
        (reinterpret_cast<uintptr_t>(lmeta + 2 * lmax) + 7) & ~uintptr_t(7)); // lmax
    double* lfac = reinterpret_cast<double*>(loff + lmax);                   // 16
    const int s = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int k0 = blockIdx.y * KC;
    const int kc = min(KC, P - k0);
    const int node0 = sub_node_off[s];
    const int nloc = sub_node_off[s + 1] - node0;
    const int lv0 = sub_lev_off[s], lv1 = sub_lev_off[s + 1];

    TS pre[NPF];
    double rv[NQ];
    int cidx[NQ][KCP];
    double cval[NQ][KCP];
    double zsv[4], zcur[4];

    // phase-A position q -> (row c of the tile, column j)
    auto pos = [&](int q, int cp, int& c, int& j) {
        if constexpr (MM::ytrans) { j = q / cp; c = q - j * cp; }
        else { c = q >> 4; j = q & 15; }
    };
    auto yidx = [&](int c, int j, int cp) { return MM::ytrans ? j * cp + c : c * 16 + j; };

    for (int q = tid; q < nloc; q += kRasThreads)
        lgn[q] = gnode[node0 + q] | (owned[node0 + q] ? int32_t(0x80000000u) : 0);
    for (int q = tid; q < lv1 - lv0; q += kRasThreads) {
        lmeta[2 * q] = lev_start[lv0 + q];
        lmeta[2 * q + 1] = lev_size[lv0 + q];
        loff[q] = sinv_off[lv0 + q];
    }
    if constexpr (!SETUP) {
        if (tid < 16) lfac[tid] = tid < kc ? omega / afact[k0 + tid] : 0.0;
    }
    auto LST = [&](int lv) { return lmeta[2 * (lv - lv0)]; };
    auto LSZ = [&](int lv) { return lmeta[2 * (lv - lv0) + 1]; };
    auto LOF = [&](int lv) { return loff[lv - lv0]; };
    auto gid = [&](int row) { return lgn[row] & 0x7fffffff; };

    auto prefetch_S = [&](int lv) {
        const int b = LSZ(lv);
        const int64_t off = LOF(lv);
        const int rp = rp_of(b), cp = cp_of(b);
#pragma unroll
        for (int p = 0; p < NPF; ++p) {
            const int q = tid + p * kRasThreads;
            if (q < rp * cp) {
                const int r = q / cp, c = q - r * cp;
                pre[p] = (r < b && c < b) ? sinv[off + (int64_t)r * b + c] : TS(0);
            }
        }
    };
    auto commit_S = [&](int lv) {
        const int b = LSZ(lv);
        const int rp = rp_of(b), cp = cp_of(b);
#pragma unroll
        for (int p = 0; p < NPF; ++p) {
            const int q = tid + p * kRasThreads;
            if (q < rp * cp) Sb[q] = pre[p];
        }
    };
    auto prefetch_rows = [&](int lv, bool fwd) {
        const int st = LST(lv), b = LSZ(lv);
        const int cp = cp_of(b);
        const int32_t* ci = fwd ? prev_idx : next_idx;
        const double* cv = fwd ? prev_val : next_val;
#pragma unroll
        for (int o = 0; o < NQ; ++o) {
            const int q = tid + o * kRasThreads;
            int c, j;
            pos(q, cp, c, j);
            if (q < cp * 16 && c < b && j < kc) {
                const int row = st + c;
                if constexpr (SETUP) {
                    if (fwd) rv[o] = (row == qbase + k0 + j) ? 1.0 : 0.0;   // identity columns
                } else {
                    if (fwd) rv[o] = R[(size_t)gid(row) * P + k0 + j];
                }
#pragma unroll
                for (int e = 0; e < KCP; ++e) {
                    cidx[o][e] = ci[(size_t)(node0 + row) * kCouple + e];
                    cval[o][e] = cv[(size_t)(node0 + row) * kCouple + e];
                }
            }
        }
        if (!fwd) {
            const int rt = rp_of(b) / 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * wave + MM::row_of(lane, v), j = lane & 15;
                if (wave < rt && r < b && j < kc) zsv[v] = zs[(size_t)(node0 + st + r) * P + k0 + j];
            }
        }
    };
    // offset of local row `row`, column k0 + k in Z if the row is owned, else -1
    auto out_index = [&](int row, int k) -> int64_t {
        const int g = lgn[row];
        return g < 0 ? (int64_t)(g & 0x7fffffff) * P + k0 + k : -1;
    };
    auto store_out = [&](int64_t o, int k, double x, double zold) {
        const double v = x * lfac[k];
        Z[o] = beta != 0.0 ? fma(beta, zold, v) : v;
    };
    auto write_out = [&](int row, int k, double x) {
        const int g = lgn[row];
        if constexpr (SETUP) {
            const int q = qbase + k0 + k;
            if (g < 0 && q < nloc)
                ainv[ainv_off[s] + (int64_t)own_pos[node0 + row] * ainv_ld[s] + q] = x;
            return;
        }
        if (g < 0) {
            const size_t o = (size_t)(g & 0x7fffffff) * P + k0 + k;
            const double v = x * lfac[k];
            Z[o] = beta != 0.0 ? fma(beta, Z[o], v) : v;
        }
    };
    // phase B: S_l^{-1} (wave's row tile) * Y on the matrix cores
    auto product = [&](int b) -> typename MM::Acc {
        const int nk = cp_of(b) / KS;
        const int cp = cp_of(b);
        typename MM::Acc acc = MM::zero();
#pragma unroll
        for (int t = 0; t < NK; ++t)
            if (t < nk) acc = MM::step(Sb, cp, Y, t * KS, lane, wave, acc);
        return acc;
    };

    // ---------------- forward sweep
    lds_barrier();                               // lgn ready
    prefetch_S(lv0);
    prefetch_rows(lv0, true);
    for (int lv = lv0; lv < lv1; ++lv) {
        const int st = LST(lv), b = LSZ(lv);
        const int cp = cp_of(b);
        commit_S(lv);
#pragma unroll
        for (int o = 0; o < NQ; ++o) {
            const int q = tid + o * kRasThreads;
            if (q < cp * 16) {
                int c, j;
                pos(q, cp, c, j);
                double y = 0.0;
                if (c < b && j < kc) {
                    y = rv[o];
                    if (lv > lv0) {
#pragma unroll
                        for (int e = 0; e < KCP; ++e)
                            if (cidx[o][e] >= 0) y = fma(-cval[o][e], Zp[cidx[o][e] * 16 + j], y);
                    }
                }
                Y[yidx(c, j, cp)] = MM::conv(y);
            }
        }
        lds_barrier();
        if (lv + 1 < lv1) {
            prefetch_S(lv + 1);
            prefetch_rows(lv + 1, true);
        }
        if (wave < rp_of(b) / 16) {
            const auto acc = product(b);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * wave + MM::row_of(lane, v), j = lane & 15;
                if (r < b && j < kc) {
                    const double z = (double)acc[v];
                    Zc[r * 16 + j] = z;
                    zs[(size_t)(node0 + st + r) * P + k0 + j] = z;
                }
            }
        }
        lds_barrier();
        double* t = Zp; Zp = Zc; Zc = t;
    }

    // ---------------- backward sweep: Zp holds x of the last level
    {
        const int lv = lv1 - 1;
        const int st = LST(lv), b = LSZ(lv);
        if constexpr (SETUP) {
            for (int q = tid; q < b * 16; q += kRasThreads) {
                const int r = q >> 4, j = q & 15;
                if (j < kc) write_out(st + r, j, Zp[r * 16 + j]);
            }
        } else {
            // Z may be accumulated into: every old value is read before the
            // first store, so the loads do not wait behind the stores
            constexpr int NO = (BM * 16 + kRasThreads - 1) / kRasThreads;
            int64_t zo[NO];
            double zold[NO];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const int q = tid + o * kRasThreads, r = q >> 4, j = q & 15;
                zo[o] = (r < b && j < kc) ? out_index(st + r, j) : -1;
                zold[o] = (beta != 0.0 && zo[o] >= 0) ? Z[zo[o]] : 0.0;
            }
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const int q = tid + o * kRasThreads, r = q >> 4, j = q & 15;
                if (zo[o] >= 0) store_out(zo[o], j, Zp[r * 16 + j], zold[o]);
            }
        }
    }
    if (lv1 - 2 < lv0) return;
    prefetch_S(lv1 - 2);
    prefetch_rows(lv1 - 2, false);
    double* Xn = Zp;
    double* Xc = Zc;
    for (int lv = lv1 - 2; lv >= lv0; --lv) {
        const int st = LST(lv), b = LSZ(lv);
        const int cp = cp_of(b);
        commit_S(lv);
#pragma unroll
        for (int o = 0; o < NQ; ++o) {
            const int q = tid + o * kRasThreads;
            if (q < cp * 16) {
                int c, j;
                pos(q, cp, c, j);
                double t = 0.0;
                if (c < b && j < kc) {
#pragma unroll
                    for (int e = 0; e < KCP; ++e)
                        if (cidx[o][e] >= 0) t = fma(cval[o][e], Xn[cidx[o][e] * 16 + j], t);
                }
                Y[yidx(c, j, cp)] = MM::conv(t);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) zcur[v] = zsv[v];
        lds_barrier();
        if (lv - 1 >= lv0) {
            prefetch_S(lv - 1);
            prefetch_rows(lv - 1, false);
        }
        if (wave < rp_of(b) / 16) {
            // old values of the owned outputs are fetched before the product
            int64_t zo[4];
            double zold[4];
            if constexpr (!SETUP) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * wave + MM::row_of(lane, v), j = lane & 15;
                    zo[v] = (r < b && j < kc) ? out_index(st + r, j) : -1;
                    zold[v] = (beta != 0.0 && zo[v] >= 0) ? Z[zo[v]] : 0.0;
                }
            }
            const auto acc = product(b);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * wave + MM::row_of(lane, v), j = lane & 15;
                if (r < b && j < kc) {
                    const double x = zcur[v] - (double)acc[v];
                    Xc[r * 16 + j] = x;
                    if constexpr (SETUP)
                        write_out(st + r, j, x);
                    else if (zo[v] >= 0)
                        store_out(zo[v], j, x, zold[v]);
                }
            }
        }
        lds_barrier();
        double* t2 = Xn; Xn = Xc; Xc = t2;
    }
}

// ---------------------------------------------------------------- dense path
// Right-hand sides of all subdomains, transposed and converted:
// xg[s][n][q] = R[gnode(s, q)][n] (zero for n >= P and q >= nloc).  One
// work-group per (subdomain, 64 local nodes), staged through LDS so that the
// reads of R and the writes of xg are both contiguous.
template <class TS>
__global__ __launch_bounds__(256) void dense_gather_kernel(
    int P, int Pp, const int32_t* __restrict__ sub_node_off, const int32_t* __restrict__ gnode,
    const int32_t* __restrict__ ld, const int64_t* __restrict__ xoff, const double* __restrict__ R,
    TS* __restrict__ xg) {
    __shared__ double tile[64][65];
    const int s = blockIdx.x, q0 = blockIdx.y * 64;
    const int node0 = sub_node_off[s], nloc = sub_node_off[s + 1] - node0;
    if (q0 >= nloc) return;
    const int nq = min(64, nloc - q0);
    const int tid = threadIdx.x;
    const int lds_s = ld[s];
    TS* out = xg + xoff[s];
    for (int n0 = 0; n0 < P; n0 += 64) {
        const int nn = min(64, P - n0);
        // consecutive threads read consecutive columns of a node, then the next
        // node: every lane carries a value, and nodes with consecutive global
        // numbers give contiguous reads
        for (int e = tid; e < nq * nn; e += 256) {
            const int qq = e / nn, nl = e - qq * nn;
            tile[qq][nl] = R[(size_t)gnode[node0 + q0 + qq] * P + n0 + nl];
        }
        __syncthreads();
        for (int e = tid; e < nn * 64; e += 256) {
            const int nl = e >> 6, qq = e & 63;
            if (qq < nq) out[(size_t)(n0 + nl) * lds_s + q0 + qq] = Mma<TS>::conv(tile[qq][nl]);
        }
        __syncthreads();
    }
    (void)Pp;
}

// Z[owned] = beta Z[owned] + omega / n! * (Ainv_s X_s)[own rows]: one wave per
// 64 owned rows (MT = 4 row tiles of 16) and all P columns (NT tiles of 16),
// K = local nodes.  The sum over k runs in any order as long as the A and B
// operands agree, so in each super-step of 2 MFMA k-steps lane group g takes
// the 32 bytes at offset 32 g of the 128-byte row segment (whole lines of X).
// The inverse is stored tile by tile in exactly that load order (below), so
// each load instruction of a wave reads 1 KB of consecutive bytes and a wave
// streams each of its row tiles from one contiguous range.  Every
// right-hand-side fragment loaded serves the MT row tiles.
constexpr int kDenseRowChoices[] = {64, 32};   // rows per wave
constexpr int kDenseLd = 64;         // local-node padding of the stored rows

// Tiled storage of one subdomain's inverse rows, for entries of TS (KL =
// 16 / sizeof(TS) per 16-byte load, KSUP = 8 KL per super-step).  Rows come
// in blocks of four row tiles (64 rows, n_own padded to a multiple of 64):
// row tile rt (rows 16 rt .. 16 rt + 15), super-step ks, half h and lane
// l = i + 16 g hold the KL entries of row 16 rt + i at columns
// ks KSUP + 2 KL g + h KL + (0 .. KL-1), at element offset
// (rt / 4) 64 ld + (((2 ks + h) 4 + rt % 4) 64 + l) KL.  A wave that takes
// the four tiles of a block reads one contiguous 4 KB per half super-step.
// Rows past n_own are zero.
constexpr int kTileBlock = 4;                 // row tiles per stored block
template <class TS>
__global__ __launch_bounds__(256) void tile_dense_kernel(
    const int32_t* __restrict__ nown, const int32_t* __restrict__ ld,
    const int64_t* __restrict__ aoff, const int64_t* __restrict__ toff,
    const double* __restrict__ rows, TS* __restrict__ out) {
    constexpr int KL = 16 / sizeof(TS);
    const int s = blockIdx.x, rt = blockIdx.y;
    const int no = nown[s];
    if (16 * rt >= (no + 63) / 64 * 64) return;
    const int L = ld[s];
    const double* src = rows + aoff[s];
    TS* dst = out + toff[s] + (int64_t)(rt / kTileBlock) * 64 * L + (rt % kTileBlock) * 64 * KL;
    for (int o = threadIdx.x; o < 16 * L; o += 256) {
        const int e = o % KL, l = (o / KL) & 63, h = (o / (64 * KL)) & 1, ks = o / (128 * KL);
        const int row = 16 * rt + (l & 15);
        const int col = ks * 8 * KL + 2 * KL * (l >> 4) + h * KL + e;
        dst[(int64_t)(o / (64 * KL)) * kTileBlock * 64 * KL + o % (64 * KL)] =
            Mma<TS>::conv(row < no ? src[(int64_t)row * L + col] : 0.0);
    }
}

// One 16-byte A fragment times one 16-byte B fragment on the matrix cores
// (one MFMA k-step of 32 BF16, four of 4 FP32 or two of 4 FP64 entries).
template <class TS>
__device__ inline void dense_mma(typename Mma<TS>::Acc& acc, const uint4& av, const uint4& bv) {
    if constexpr (sizeof(TS) == 2) {
        sg_bf8 a, bb;
        __builtin_memcpy(&a, &av, 16);
        __builtin_memcpy(&bb, &bv, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
    } else if constexpr (sizeof(TS) == 4) {
        float a[4], bb[4];
        __builtin_memcpy(a, &av, 16);
        __builtin_memcpy(bb, &bv, 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], bb[u], acc, 0, 0, 0);
    } else {
        double a[2], bb[2];
        __builtin_memcpy(a, &av, 16);
        __builtin_memcpy(bb, &bv, 16);
#pragma unroll
        for (int u = 0; u < 2; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[u], acc, 0, 0, 0);
    }
}

// Z[own_gnode[r]][n] = beta Z[..] + omega acc / n! for the wave's rows
// r0 .. r0 + 16 MT - 1 (those below no) and n < P.  Z may be accumulated
// into: per row tile, the old values are all read before the first store, so
// the loads do not wait behind each store.
template <class TS, int NT, int MT>
__device__ inline void dense_epilogue(const typename Mma<TS>::Acc (&acc)[MT][NT], int P, int r0, int no,
                                      int lane, const int32_t* __restrict__ own_gnode,
                                      const double* __restrict__ afact, double* Z, double omega,
                                      double beta) {
    const int i = lane & 15;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        int64_t zo[4];
        double zold[NT][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * m + Mma<TS>::row_of(lane, v);
            zo[v] = r < no ? (int64_t)own_gnode[r] * P : -1;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int n = 16 * t + i;
                zold[t][v] = (beta != 0.0 && zo[v] >= 0 && n < P) ? Z[zo[v] + n] : 0.0;
            }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int n = 16 * t + i;
                if (zo[v] >= 0 && n < P) {
                    const double val = omega * (double)acc[m][t][v] / afact[n];
                    Z[zo[v] + n] = beta != 0.0 ? fma(beta, zold[t][v], val) : val;
                }
            }
    }
}

template <class TS, int NT, int kDenseRows>
__global__ __launch_bounds__(256) void dense_apply_kernel(
    int P, const int32_t* __restrict__ blk_sub, const int32_t* __restrict__ blk_row0,
    const int32_t* __restrict__ nown, const int32_t* __restrict__ ld,
    const int64_t* __restrict__ toff, const int64_t* __restrict__ xoff,
    const int64_t* __restrict__ own_off, const int32_t* __restrict__ own_gnode,
    const TS* __restrict__ ainv, const TS* __restrict__ xg, const double* __restrict__ afact,
    double* Z, double omega, double beta) {
    using Acc = typename Mma<TS>::Acc;
    constexpr int MT = kDenseRows / 16;
    constexpr int KL = 16 / sizeof(TS);          // elements per 16-byte load
    constexpr int KSUP = 8 * KL;                 // elements per super-step (128 bytes per row)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const int s = blk_sub[b];
    const int r0 = blk_row0[b] + kDenseRows * wave;
    const int no = nown[s];
    if (r0 >= no) return;
    const int L = ld[s];
    const int i = lane & 15, g = lane >> 4;
    // r0 is a multiple of 16 MT: the wave's row tiles lie in one stored block
    // (tiles past n_own are zero)
    const TS* A[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int rt = (r0 >> 4) + m;
        A[m] = ainv + toff[s] + (int64_t)(rt / kTileBlock) * 64 * L +
               (rt % kTileBlock) * 64 * KL + lane * KL;
    }
    const TS* X = xg + xoff[s] + (int64_t)i * L + 2 * KL * g;
    Acc acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = Mma<TS>::zero();
    // two register buffers: the loads of super-step k + 1 are in flight while
    // the products of super-step k run
    uint4 av[2][MT][2], bv[2][NT][2];
    auto load = [&](int buf, int k) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            av[buf][m][0] = *reinterpret_cast<const uint4*>(A[m] + 16 * kTileBlock * k);
            av[buf][m][1] =
                *reinterpret_cast<const uint4*>(A[m] + 16 * kTileBlock * k + kTileBlock * 64 * KL);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bv[buf][t][0] = *reinterpret_cast<const uint4*>(X + (int64_t)16 * t * L + k);
            bv[buf][t][1] = *reinterpret_cast<const uint4*>(X + (int64_t)16 * t * L + k + KL);
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) dense_mma<TS>(acc[m][t], av[buf][m][h], bv[buf][t][h]);
    };
    load(0, 0);
    int k = 0;
    for (; k + 2 * KSUP <= L; k += 2 * KSUP) {
        load(1, k + KSUP);
        compute(0);
        if (k + 2 * KSUP < L) load(0, k + 2 * KSUP);
        compute(1);
    }
    if (k < L) compute(0);          // L / KSUP odd: the last super-step is in buffer 0
    dense_epilogue<TS, NT, MT>(acc, P, r0, no, lane, own_gnode + own_off[s], afact, Z, omega, beta);
}

// Fused dense apply: one work-group of kFusedWaves waves per (subdomain,
// kFusedRows owned rows).  The work-group gathers the subdomain's right-hand
// sides from R into LDS itself, converted and already in the order in which
// the lanes take their B fragments ([super-step][column tile][half][lane],
// 16 bytes each), so the separate gather pass and the re-reads of the
// gathered copy through L2 disappear.  After one barrier each wave streams
// its 64 rows of the tiled inverse with B read from LDS and no further
// barrier.
// LDS: Pp x ld entries of TS plus ld node ids.
constexpr int kFusedWaves = 16;
constexpr int kFusedRows = 64 * kFusedWaves;
constexpr int kFusedChunks = 7;   // right-hand-side chunks gathered under the stream
// column tiles whose accumulators fit the 128 registers of a 16-wave group
inline int fused_max_nt(sg_prec prec) { return prec == SG_FP64 ? 1 : 3; }
// Output mixing of the Kronecker local solves in the fused path (POST): after
// the stream Gt^{-1} is staged in LDS, every wave dumps 32 of its 64 rows of
// accumulators to its own LDS slice (row stride Pp + 1), two lanes per row
// multiply it by Gt^{-1} (half the columns each) and write it back, and the
// wave stores the slice to Z with consecutive lanes on consecutive entries
// of the flattened rows; then the other 32 rows.
// After them, per wave, the global node of each of its 64 rows and that
// node's coarse owner (two int32 each).
inline size_t dense_post_lds(int P, int Pp, size_t acc_bytes) {
    return ((size_t)kFusedWaves * 32 * (Pp + 1) + (size_t)P * Pp) * acc_bytes +
           (size_t)kFusedWaves * 128 * sizeof(int32_t);
}

// STORE: 0 = stores from the matrix-core layout (dense_epilogue); 1 = the
// output mixing by Gt^{-1} (Kronecker local solves); 2 = the same row-slice
// store with the division by alpha! (mean-based local solves), bit-identical
// to 0.
template <class TS, int NT, int STORE>
__global__ __launch_bounds__(64 * kFusedWaves) void dense_fused_kernel(
    int P, const int32_t* __restrict__ blk_sub, const int32_t* __restrict__ blk_row0,
    const int32_t* __restrict__ nown, const int32_t* __restrict__ ld,
    const int32_t* __restrict__ sub_node_off, const int32_t* __restrict__ gnode,
    const int64_t* __restrict__ toff, const int64_t* __restrict__ own_off,
    const int32_t* __restrict__ own_gnode, const TS* __restrict__ ainv,
    const double* __restrict__ R, const double* __restrict__ afact, double* Z, double omega,
    double beta, const double* __restrict__ post, const double* __restrict__ cadd,
    const int32_t* __restrict__ cown) {
    using Acc = typename Mma<TS>::Acc;
    constexpr int MT = 4;
    constexpr int KL = 16 / sizeof(TS);
    constexpr int KSUP = 8 * KL;
    constexpr int Pp = 16 * NT;
    constexpr int kThreads = 64 * kFusedWaves;
    extern __shared__ uint4 lds_b[];
    // the wave index is uniform: the row tiles and their base addresses stay
    // in scalar registers, each lane adds one offset
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = blk_sub[blockIdx.x];
    const int r0 = blk_row0[blockIdx.x] + 64 * wave;
    const int no = nown[s];
    const int L = ld[s];
    const int nks = L / KSUP;
    const int node0 = sub_node_off[s], nloc = sub_node_off[s + 1] - node0;
    const bool active = r0 < no;
    // the wave's four row tiles are one stored block (r0 is a multiple of
    // 64): a scalar base plus one 32-bit byte offset per lane (a block holds
    // 64 ld entries, well below 4 GB)
    static_assert(MT == kTileBlock, "one wave streams one block of row tiles");
    const char* A = reinterpret_cast<const char*>(ainv + toff[s] + (int64_t)(r0 >> 6) * 64 * L);
    // the stream runs in half super-steps (one MFMA k-step pair for BF16):
    // half j of row tile m is the 1 KB at byte 1024 (4 j + m), and its B
    // fragments are piece (2 (j / 2) NT + 2 t + j % 2) 64 + lane
    constexpr bool kBurst = std::is_same<TS, float>::value;
    uint4 av[kBurst ? 2 : 3][MT];
    auto aload = [&](int slot, int j) {
        const uint32_t off = (uint32_t)lane * 16u + (uint32_t)j * (1024u * MT);
#pragma unroll
        for (int m = 0; m < MT; ++m)
            av[slot][m] = *reinterpret_cast<const uint4*>(A + off + 1024u * m);
    };
    const int nh = 2 * nks;   // >= 2
    if (active) {             // the first half-steps of the ring load during the gather
        aload(0, 0);
        aload(1, 1);
        if constexpr (!kBurst) {
            if (nh > 2) aload(2, 2);
        }
    }
    // The right-hand sides arrive in chunks of CS super-steps (a multiple of
    // three, so that chunk borders fall on the three-slot ring below; the
    // FP32 form's two-slot ring needs only the even count of half-steps).  Entry
    // e of a chunk is local node q0 + e / P, column e % P: consecutive threads
    // read consecutive entries of a node's row of R; padded nodes are zero.
    // Only chunks c (streamed) and c + 1 (gathered) are live at once, so the
    // LDS holds a ring of two chunks: super-step ks sits at ks mod 2 CS.
    const int CS = 3 * ((nks + 3 * kFusedChunks - 1) / (3 * kFusedChunks));
    const int nchunks = (nks + CS - 1) / CS;
    const int ring = min(nks, 2 * CS);        // super-steps held
    // node ids after the B pieces
    int32_t* ids = reinterpret_cast<int32_t*>(lds_b + (size_t)ring * NT * 128);
    for (int q = tid; q < nloc; q += kThreads) ids[q] = gnode[node0 + q];
    TS* bsh = reinterpret_cast<TS*>(lds_b);
    // LDS slot of entry (local node q, column n)
    auto slot = [&](int q, int n) {
        const int ks = q / KSUP, w = q - ks * KSUP;
        const int g = w / (2 * KL), h = (w / KL) & 1, el = w % KL;
        return ((((ks % (2 * CS)) * NT + (n >> 4)) * 2 + h) * 64 + (n & 15) + 16 * g) * KL + el;
    };
    // zeros in the padded columns P .. Pp - 1 of the ring (no chunk's gather
    // writes them)
    const int npad = Pp - P;
    for (int e = tid; e < ring * KSUP * npad; e += kThreads) {
        const int q = e / npad;
        bsh[slot(q, P + e - q * npad)] = Mma<TS>::conv(0.0);
    }
    __syncthreads();
    auto chunk_count = [&](int c) { return (min((c + 1) * CS * KSUP, L) - c * CS * KSUP) * P; };
    auto fetch = [&](int c, int e) {
        const int q = c * CS * KSUP + e / P;
        return q < nloc ? R[(int64_t)ids[q] * P + (e - (e / P) * P)] : 0.0;
    };
    auto put = [&](int c, int e, double v) {
        const int q = c * CS * KSUP + e / P;
        bsh[slot(q, e - (e / P) * P)] = Mma<TS>::conv(v);
    };
    {   // chunk 0 in full, U loads in flight per thread
        constexpr int U = 8;
        const int cnt = chunk_count(0);
        for (int base = tid; base < cnt; base += U * kThreads) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = base + u * kThreads;
                v[u] = e < cnt ? fetch(0, e) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (base + u * kThreads < cnt) put(0, base + u * kThreads, v[u]);
        }
    }
    __syncthreads();
    Acc acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = Mma<TS>::zero();
    auto compute = [&](int slot_, int j) {
        const int pb = (2 * ((j >> 1) % (2 * CS)) * NT + (j & 1)) * 64 + lane;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint4 b = lds_b[pb + 128 * t];
#pragma unroll
            for (int m = 0; m < MT; ++m) dense_mma<TS>(acc[m][t], av[slot_][m], b);
        }
    };
    // Two forms of the stream, chosen by measurement on config 1: for FP32
    // the gather in one burst per chunk (apply 430 -> 393 us after a cache
    // flush); for BF16 the per-half-step gather (the burst form measured
    // 186 -> 191 us back to back there), which FP64 keeps as well.
    if constexpr (kBurst) {
        // Entry e < chunk_count(c) of chunk c, read whatever the data: the node
        // index is clamped and padded nodes are zeroed afterwards.
        auto fetch_clamped = [&](int c, int e) {
            const int q = c * CS * KSUP + e / P;
            const double v = R[(int64_t)ids[min(q, nloc - 1)] * P + (e - (e / P) * P)];
            return q < nloc ? v : 0.0;
        };
        // The stream of chunk c.  At its start every thread fetches its first
        // GB entries of chunk c + 1 (entries tid, tid + 1024, ...) into
        // registers; it stores them to LDS at the chunk's end, fetches what is
        // left of the chunk, and a barrier publishes it.  In between, half-step
        // jj runs the products of jj (A from ring slot jj % 2, B from LDS) and
        // the A loads of half-step jj + 2 into the slot just used.  Every
        // half-step issues the same loads whatever the data (addresses clamped,
        // no load on one path only), so the compiler's count of loads in flight
        // stays exact: the products of jj wait for the loads of jj (and those
        // before), and the next half-step's loads stay in flight; the gathered
        // entries are waited for once, at the chunk's end.  (Where a
        // load is issued on one path only, the count is lost and every wait
        // becomes a wait for all loads.)  Waves past the subdomain's rows (ACT
        // false) only gather.
        constexpr int GB = 7;
        auto stream = [&](auto act, auto gather, int c) {
            constexpr bool ACT = decltype(act)::value, GATHER = decltype(gather)::value;
            const int j0 = 2 * c * CS, j1 = min(2 * (c + 1) * CS, nh);
            const int cn = GATHER ? chunk_count(c + 1) : 0;
            double gv[GB];
            if constexpr (GATHER) {
#pragma unroll
                for (int u = 0; u < GB; ++u)
                    gv[u] = fetch_clamped(c + 1, min(tid + u * kThreads, cn - 1));
            }
            auto step = [&](int r, int jj) {
                if constexpr (ACT) {
                    compute(r, jj);
                    aload(r, min(jj + 2, nh - 1));
                }
            };
            // j0 and j1 - j0 are even: ring slot jj % 2 is r
            for (int j = j0; j < j1; j += 2) {
                step(0, j);
                step(1, j + 1);
            }
            if constexpr (GATHER) {
                // a thread past the chunk's entries fetched entry cn - 1 and
                // stores that same value again
#pragma unroll
                for (int u = 0; u < GB; ++u) put(c + 1, min(tid + u * kThreads, cn - 1), gv[u]);
                for (int e = tid + GB * kThreads; e < cn; e += kThreads) put(c + 1, e, fetch(c + 1, e));
                lds_barrier();   // the ring's A loads stay in flight across it
            }
        };
        const std::true_type yes{};
        const std::false_type no_{};
        if (active) {
            for (int c = 0; c + 1 < nchunks; ++c) stream(yes, yes, c);
            stream(yes, no_, nchunks - 1);
        } else {
            for (int c = 0; c + 1 < nchunks; ++c) stream(no_, yes, c);
            stream(no_, no_, nchunks - 1);
        }
    } else {
        // While chunk c streams, every thread (active wave or not) fetches two
        // entries of chunk c + 1 per half-step and stores the two it fetched one
        // half-step earlier; what is left of chunk c + 1 is fetched at the end of
        // chunk c, then a barrier publishes it.  A wave's A stream is the ring of
        // three half-steps: slot j % 3 is refilled three halves ahead once its
        // products are issued.
        for (int c = 0; c < nchunks; ++c) {
            const int j0 = 2 * c * CS, j1 = min(2 * (c + 1) * CS, nh);
            const int cn = c + 1 < nchunks ? chunk_count(c + 1) : 0;
            int ge = tid;                      // next entry of chunk c + 1 for this thread
            double gv[2] = {0.0, 0.0};
            int ga[2] = {-1, -1};              // entries fetched one half-step ago
            auto gather_step = [&]() {
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (ga[u] >= 0) put(c + 1, ga[u], gv[u]);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    ga[u] = ge < cn ? ge : -1;
                    if (ga[u] >= 0) gv[u] = fetch(c + 1, ge);
                    ge += kThreads;
                }
            };
            for (int j = j0; j < j1; j += 3) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int jj = j + r;
                    if (jj < j1) {
                        // the gather's stores wait for its loads of the previous
                        // half-step and for every load issued before them; the A
                        // loads issued after those stay in flight
                        if (active) compute(r, jj);
                        if (cn > 0) gather_step();
                        if (active && jj + 3 < nh) aload(r, jj + 3);
                    }
                }
            }
            if (cn > 0) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (ga[u] >= 0) put(c + 1, ga[u], gv[u]);
                for (; ge < cn; ge += kThreads) put(c + 1, ge, fetch(c + 1, ge));
                lds_barrier();   // the ring's A loads stay in flight across it
            }
        }
    }
    if constexpr (STORE != 0) {
        using AT = typename std::conditional<std::is_same<TS, double>::value, double, float>::type;
        constexpr int RS = Pp + 1;          // odd row stride: conflict-free row reads
        constexpr int JH = Pp / 2;          // columns per lane (two lanes per row)
        constexpr int UB = 8;               // stores per batch, their loads issued together
        __syncthreads();                    // every wave has streamed: the LDS is free
        // Gt^{-1} after the row slices, in the accumulator precision
        AT* ps = reinterpret_cast<AT*>(lds_b) + (size_t)kFusedWaves * 32 * RS;
        int32_t* info = reinterpret_cast<int32_t*>(ps + (STORE == 1 ? P * Pp : 0)) + wave * 128;
        if (active) {   // this wave's rows: global node, and its coarse owner
            const int row = r0 + lane;
            const int gn = row < no ? own_gnode[own_off[s] + row] : 0;
            info[lane] = gn;
            info[64 + lane] = (cadd && row < no) ? cown[gn] : 0;
        }
        if (STORE == 1) {
            for (int q = tid; q < P * Pp; q += kThreads) ps[q] = (AT)post[q];
            __syncthreads();
        }
        if (!active) return;
        AT* rb = reinterpret_cast<AT*>(lds_b) + (size_t)wave * 32 * RS;
        const int i = lane & 15;
        const int row = lane & 31, j0 = (lane >> 5) * JH;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        rb[(16 * m + Mma<TS>::row_of(lane, v)) * RS + 16 * t + i] =
                            acc[2 * hf + m][t][v];
            if constexpr (STORE == 1 && std::is_same<AT, float>::value) {
                // the slice times Gt^{-1} on the matrix cores: 32 x Pp by
                // P x Pp in k-steps of 4 (A from the slice, whose columns
                // P .. Pp - 1 are zero; B rows past P read as zero), then the
                // products written over the slice; the LDS runs a wave's
                // instructions in order, so every read precedes the writes
                using Acc = typename Mma<float>::Acc;
                Acc z[2][NT];
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int t = 0; t < NT; ++t) z[m][t] = Mma<float>::zero();
                for (int k0 = 0; k0 < P; k0 += 4) {
                    const int kk = k0 + (lane >> 4);
                    float a[2], b[NT];
#pragma unroll
                    for (int m = 0; m < 2; ++m) a[m] = rb[(16 * m + i) * RS + kk];
#pragma unroll
                    for (int t = 0; t < NT; ++t) b[t] = kk < P ? ps[kk * Pp + 16 * t + i] : 0.f;
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            z[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[t], z[m][t], 0, 0, 0);
                }
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            rb[(16 * m + Mma<float>::row_of(lane, v)) * RS + 16 * t + i] = z[m][t][v];
            } else if constexpr (STORE == 1) {
                AT z[JH];
#pragma unroll
                for (int j = 0; j < JH; ++j) z[j] = AT(0);
                for (int k = 0; k < P; ++k) {
                    const AT xk = rb[row * RS + k];
                    const AT* pk = ps + k * Pp + j0;
#pragma unroll
                    for (int j = 0; j < JH; ++j) z[j] = fma(xk, pk[j], z[j]);
                }
                // both lanes of a row have read it (the LDS runs a wave's
                // instructions in order) before either overwrites its half
#pragma unroll
                for (int j = 0; j < JH; ++j) rb[row * RS + j0 + j] = z[j];
            }
            // entry e of the slice is row e / P, column e % P; the old values
            // of a batch (Z and the coarse correction) are loaded before any
            // of its stores, so they are in flight together
            const int rbase = 32 * hf;
            const int ne = min(32, no - (r0 + rbase)) * P;
            for (int e0 = lane; e0 < ne; e0 += UB * 64) {
                double zold[UB], cv[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = e0 + 64 * u;
                    const int rr = e / P, c = e - rr * P;
                    zold[u] = 0.0;
                    cv[u] = 0.0;
                    if (beta != 0.0 && e < ne) {
                        zold[u] = Z[(int64_t)info[rbase + rr] * P + c];
                        // z2 = z1 + Z e_c formed here, as the prolongation would
                        if (cadd) cv[u] = cadd[(int64_t)info[64 + rbase + rr] * P + c];
                    }
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = e0 + 64 * u;
                    if (e < ne) {
                        const int rr = e / P, c = e - rr * P;
                        const double val = STORE == 1 ? omega * (double)rb[rr * RS + c]
                                                      : omega * (double)rb[rr * RS + c] / afact[c];
                        const double zo = cadd ? zold[u] + cv[u] : zold[u];
                        Z[(int64_t)info[rbase + rr] * P + c] = beta != 0.0 ? fma(beta, zo, val) : val;
                    }
                }
            }
        }
        return;
    }
    if (!active) return;
    dense_epilogue<TS, NT, MT>(acc, P, r0, no, lane, own_gnode + own_off[s], afact, Z, omega, beta);
}

// LDS of the fused path: the ring of two right-hand-side chunks (as the
// kernel sizes its chunks for the widest subdomain) plus the node ids.
inline size_t dense_fused_lds(size_t entry_bytes, int Pp, int ld_max) {
    const int ksup = 8 * (int)(16 / entry_bytes);
    const int nks = ld_max / ksup;
    const int cs = 3 * ((nks + 3 * kFusedChunks - 1) / (3 * kFusedChunks));
    const int ring = std::min(nks, 2 * cs);
    return (size_t)Pp * ring * ksup * entry_bytes + (size_t)ld_max * 4;
}

}  // namespace

void ras_dense_apply(const sg_ras* r, const double* R, double* Z, double omega, double beta,
                     hipStream_t s, bool post, const double* cadd, const int32_t* cown) {
    int maxn = 0;
    for (size_t q = 0; q + 1 < r->h_sub_node_off.size(); ++q)
        maxn = std::max(maxn, r->h_sub_node_off[q + 1] - r->h_sub_node_off[q]);
    dim3 gg(r->n_sub, (maxn + 63) / 64);
    const int NT = r->Pp / 16;
    const int v = r->dense_var;
    if (v == 2) {
        SG_REQUIRE(r->fused_ok, "the fused dense RAS variant does not fit this problem");
        // the row-slice store (no mixing) where its LDS fits
        const size_t row_lds = dense_post_lds(0, r->Pp, r->prec == SG_FP64 ? 8 : 4);
        const bool row_store = !post && row_lds <= r->lds_max;
        SG_REQUIRE(!cadd || post || row_store, "the coarse correction needs the row-slice store");
#define SG_FUSED_NT(TS, BUF, N)                                                                    \
    case N:                                                                                        \
        if (post)                                                                                  \
            dense_fused_kernel<TS, N, 1><<<r->nblk[2], 64 * kFusedWaves,                           \
                                           std::max(r->fused_lds, r->post_lds), s>>>(              \
                r->P, r->blk_sub[2].p, r->blk_row0[2].p, r->nown_d.p, r->ld_d.p,                   \
                r->sub_node_off.p, r->gnode.p, r->toff_d.p, r->own_off_d.p, r->own_gnode.p, BUF,   \
                R, r->afact.p, Z, omega, beta, r->kron_post.p, cadd, cown);                        \
        else if (row_store)                                                                        \
            dense_fused_kernel<TS, N, 2><<<r->nblk[2], 64 * kFusedWaves,                           \
                                           std::max(r->fused_lds, row_lds), s>>>(                  \
                r->P, r->blk_sub[2].p, r->blk_row0[2].p, r->nown_d.p, r->ld_d.p,                   \
                r->sub_node_off.p, r->gnode.p, r->toff_d.p, r->own_off_d.p, r->own_gnode.p, BUF,   \
                R, r->afact.p, Z, omega, beta, nullptr, cadd, cown);                               \
        else                                                                                       \
            dense_fused_kernel<TS, N, 0><<<r->nblk[2], 64 * kFusedWaves, r->fused_lds, s>>>(       \
                r->P, r->blk_sub[2].p, r->blk_row0[2].p, r->nown_d.p, r->ld_d.p,                   \
                r->sub_node_off.p, r->gnode.p, r->toff_d.p, r->own_off_d.p, r->own_gnode.p, BUF,   \
                R, r->afact.p, Z, omega, beta, nullptr, nullptr, nullptr);                         \
        break;
        if (r->prec == SG_FP64) {
            switch (NT) {
                SG_FUSED_NT(double, r->ainv64.p, 1)
                default: SG_THROW(SG_ERR_UNSUPPORTED, "fused dense RAS with P=%d", r->P);
            }
        } else if (r->prec == SG_FP32) {
            switch (NT) {
                SG_FUSED_NT(float, r->ainv32.p, 1) SG_FUSED_NT(float, r->ainv32.p, 2)
                SG_FUSED_NT(float, r->ainv32.p, 3)
                default: SG_THROW(SG_ERR_UNSUPPORTED, "fused dense RAS with P=%d", r->P);
            }
        } else {
            switch (NT) {
                SG_FUSED_NT(uint16_t, r->ainv16.p, 1) SG_FUSED_NT(uint16_t, r->ainv16.p, 2)
                SG_FUSED_NT(uint16_t, r->ainv16.p, 3)
                default: SG_THROW(SG_ERR_UNSUPPORTED, "fused dense RAS with P=%d", r->P);
            }
        }
#undef SG_FUSED_NT
        HIP_LAUNCH_OK();
        return;
    }
#define SG_DENSE(TS, BUF)                                                                          \
    do {                                                                                           \
        dense_gather_kernel<TS><<<gg, 256, 0, s>>>(r->P, r->Pp, r->sub_node_off.p, r->gnode.p,      \
                                                   r->ld_d.p, r->xoff_d.p, R,                      \
                                                   reinterpret_cast<TS*>(r->xg.p));                \
        HIP_LAUNCH_OK();                                                                           \
        switch (NT) {                                                                              \
            SG_DENSE_NT(TS, BUF, 1) SG_DENSE_NT(TS, BUF, 2) SG_DENSE_NT(TS, BUF, 3)                \
            SG_DENSE_NT(TS, BUF, 4) SG_DENSE_NT(TS, BUF, 5) SG_DENSE_NT(TS, BUF, 6)                \
            SG_DENSE_NT(TS, BUF, 7) SG_DENSE_NT(TS, BUF, 8)                                        \
            default: SG_THROW(SG_ERR_UNSUPPORTED, "dense RAS with P=%d", r->P);                   \
        }                                                                                          \
        HIP_LAUNCH_OK();                                                                           \
    } while (0)
#define SG_DENSE_NT(TS, BUF, N)                                                                    \
    case N:                                                                                        \
        if (v == 0)                                                                                \
            dense_apply_kernel<TS, N, 64><<<r->nblk[v], 256, 0, s>>>(                               \
                r->P, r->blk_sub[v].p, r->blk_row0[v].p, r->nown_d.p, r->ld_d.p, r->toff_d.p,      \
                r->xoff_d.p, r->own_off_d.p, r->own_gnode.p, BUF,                                  \
                reinterpret_cast<const TS*>(r->xg.p), r->afact.p, Z, omega, beta);                 \
        else                                                                                       \
            dense_apply_kernel<TS, N, 32><<<r->nblk[v], 256, 0, s>>>(                               \
                r->P, r->blk_sub[v].p, r->blk_row0[v].p, r->nown_d.p, r->ld_d.p, r->toff_d.p,      \
                r->xoff_d.p, r->own_off_d.p, r->own_gnode.p, BUF,                                  \
                reinterpret_cast<const TS*>(r->xg.p), r->afact.p, Z, omega, beta);                 \
        break;
    if (r->prec == SG_FP64)
        SG_DENSE(double, r->ainv64.p);
    else if (r->prec == SG_FP32)
        SG_DENSE(float, r->ainv32.p);
    else
        SG_DENSE(uint16_t, r->ainv16.p);
#undef SG_DENSE_NT
#undef SG_DENSE
}

// W's rows are padded with zero columns to a multiple of kMixJ.
constexpr int kMixJ = 8;
inline int kron_wcols(int P) { return (P + kMixJ - 1) / kMixJ * kMixJ; }

// T[a, j] = sum_k R[a, k] W[k, j]: the mode mixing of the Kronecker local
// solve K_0 (x) Gt, applied ahead of the mean-based RAS (it acts per node, so
// it commutes with the restriction, the local K_0 solves and the partition of
// unity), on the FP64 matrix cores: per wave a tile of 64 nodes,
// T_tile (64 x P) = R_tile (64 x P) W (P x P) as 16 x 16 x 4 FP64 MFMA steps
// (four 16-row blocks per 16-column block, K in steps of 4).  Lane l feeds
// A[l % 16][l / 16] (the node row from LDS), B[l / 16][l % 16] (W from the
// cache) and holds D[l / 16 + 4 r][l % 16], r = 0..3 (checked with a probe
// of one non-zero B entry against lane-numbered A).  Rows of the tile
// past n and the K and column tails are zero-filled or not stored; a row of D
// depends only on its own row of A.
typedef double kmix_d4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(64) void kron_mix_mfma_kernel(int n, int P,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ R,
                                                           double* __restrict__ T) {
    extern __shared__ double Rs[];            // [64][P]
    const int a0 = blockIdx.x * 64, lane = threadIdx.x;
    const int na = min(64, n - a0), cnt = na * P;
    const double* rg = R + (int64_t)a0 * P;
    for (int q = lane; q < cnt; q += 64) Rs[q] = rg[q];
    for (int q = cnt + lane; q < 64 * P; q += 64) Rs[q] = 0.0;
    __syncthreads();
    const int Pw = (P + kMixJ - 1) / kMixJ * kMixJ;
    const int li = lane & 15, lk = lane >> 4;
    const int nk = (P + 3) / 4, ncb = (P + 15) / 16;
    double* tg = T + (int64_t)a0 * P;
    for (int cb = 0; cb < ncb; ++cb) {
        const int j = cb * 16 + li;
        kmix_d4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = kmix_d4{0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < nk; ++ks) {
            const int k = ks * 4 + lk;
            const double b = (k < P && j < P) ? W[(size_t)k * Pw + j] : 0.0;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const double av = k < P ? Rs[(rb * 16 + li) * P + k] : 0.0;
                acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[rb], 0, 0, 0);
            }
        }
        if (j < P) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int node = rb * 16 + lk + 4 * q;
                    if (node < na) tg[(size_t)node * P + j] = acc[rb][q];
                }
        }
    }
}

// The same MFMA mixing for P <= 4 NK with the A fragments of the whole tile
// loaded straight into registers (lane l: rows rb*16 + l % 16, columns
// 4 ks + l / 16), all issued before the first MFMA; D goes through an LDS
// tile so that each node row is stored contiguously.
template <int NK>
__global__ __launch_bounds__(64) void kron_mix_mfma_reg_kernel(int n, int P,
                                                               const double* __restrict__ W,
                                                               const double* __restrict__ R,
                                                               double* __restrict__ T) {
    const int a0 = blockIdx.x * 64, lane = threadIdx.x;
    const int na = min(64, n - a0);
    const int li = lane & 15, lk = lane >> 4;
    const int Pw = (P + kMixJ - 1) / kMixJ * kMixJ;
    double av[4][NK];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int m = rb * 16 + li;
        const double* rr = R + (int64_t)(a0 + m) * P;
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
            const int k = ks * 4 + lk;
            av[rb][ks] = (m < na && k < P) ? rr[k] : 0.0;
        }
    }
    const int ncb = (P + 15) / 16;
    extern __shared__ double Ts[];            // [64][P]: the tile's D, stored row-contiguous
    for (int cb = 0; cb < ncb; ++cb) {
        const int j = cb * 16 + li;
        kmix_d4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = kmix_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
            if (ks * 4 < P) {
                const int k = ks * 4 + lk;
                const double b = (k < P && j < P) ? W[(size_t)k * Pw + j] : 0.0;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb][ks], b, acc[rb], 0, 0, 0);
            }
        }
        if (j < P) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int q = 0; q < 4; ++q) Ts[(rb * 16 + lk + 4 * q) * P + j] = acc[rb][q];
        }
    }
    __syncthreads();
    double* tg = T + (int64_t)a0 * P;
    for (int q = lane; q < na * P; q += 64) tg[q] = Ts[q];
}

// The fused dense path with its row-slice store: it can also add a
// Nicolaides coarse correction (Z = Z + e_c[owner] + omega M R, beta = 1).
bool ras_can_add_coarse(const sg_ras* r) {
    if (!r->use_dense || r->dense_var != 2 || !r->fused_ok) return false;
    const bool post = r->local_mode == SG_LOCAL_KRON && r->post_ok && r->Pp == r->post_pp;
    if (post) return true;
    if (r->local_mode == SG_LOCAL_KRON) return false;
    return dense_post_lds(0, r->Pp, r->prec == SG_FP64 ? 8 : 4) <= r->lds_max;
}

void ras_apply_ex(const sg_ras* r, const double* R, double* Z, double omega, double beta,
                  hipStream_t s, const double* cadd, const int32_t* cown) {
    SG_REQUIRE(!cadd || (beta == 1.0 && ras_can_add_coarse(r)),
               "coarse correction inside the RAS needs the fused path and beta = 1");
    // the fused dense path mixes its output (Kronecker local solves)
    const bool post = r->local_mode == SG_LOCAL_KRON && r->use_dense && r->dense_var == 2 &&
                      r->post_ok && r->Pp == r->post_pp;
    if (r->local_mode == SG_LOCAL_KRON && !post) {
        const unsigned g = (unsigned)((r->n + 63) / 64);
        if (r->P <= 40)
            kron_mix_mfma_reg_kernel<10><<<g, 64, (size_t)64 * r->P * 8, s>>>(r->n, r->P, r->kron_w.p,
                                                                           R, r->kron_t.p);
        else if (r->P <= 64)
            kron_mix_mfma_reg_kernel<16><<<g, 64, (size_t)64 * r->P * 8, s>>>(r->n, r->P, r->kron_w.p,
                                                                           R, r->kron_t.p);
        else
            kron_mix_mfma_kernel<<<g, 64, (size_t)64 * r->P * 8, s>>>(r->n, r->P, r->kron_w.p, R,
                                                                     r->kron_t.p);
        HIP_LAUNCH_OK();
        R = r->kron_t.p;
    }
    if (r->use_dense) {
        ras_dense_apply(r, R, Z, omega, beta, s, post, cadd, cown);
        return;
    }
    const int nch = (r->P + kColChunk - 1) / kColChunk;
    const int KC = (r->P + nch - 1) / nch;
    dim3 grid(r->n_sub, nch);
    const int bmax = r->max_b, nmax = r->max_local;
    size_t lds = ras_apply_lds(r->prec, bmax, KC, nmax, r->max_levels);
#define SG_RAS_ARGS                                                                            \
    r->P, KC, bmax, nmax, r->max_levels, r->sub_node_off.p, r->sub_lev_off.p, r->lev_start.p, r->lev_size.p, \
        r->sinv_off.p
#define SG_RAS_TAIL                                                                           \
    r->gnode.p, r->owned.p, r->prev_idx.p, r->prev_val.p, r->next_idx.p, r->next_val.p,      \
        r->afact.p, R, Z, r->zs.p, omega, beta
    const bool small = bmax <= 40;
    const bool narrow = r->max_couple <= 2;
    const bool wide = r->max_couple > 4;
#define SG_RAS_GO(TS, PTR)                                                                      \
    do {                                                                                        \
        if (narrow && small)                                                                    \
            ras_apply_kernel<TS, 2, 40><<<grid, kRasThreads, lds, s>>>(SG_RAS_ARGS, PTR, SG_RAS_TAIL); \
        else if (narrow)                                                                        \
            ras_apply_kernel<TS, 2, 64><<<grid, kRasThreads, lds, s>>>(SG_RAS_ARGS, PTR, SG_RAS_TAIL); \
        else if (wide)                                                                          \
            ras_apply_kernel<TS, 8, 64><<<grid, kRasThreads, lds, s>>>(SG_RAS_ARGS, PTR, SG_RAS_TAIL); \
        else if (small)                                                                         \
            ras_apply_kernel<TS, 4, 40><<<grid, kRasThreads, lds, s>>>(SG_RAS_ARGS, PTR, SG_RAS_TAIL); \
        else                                                                                    \
            ras_apply_kernel<TS, 4, 64><<<grid, kRasThreads, lds, s>>>(SG_RAS_ARGS, PTR, SG_RAS_TAIL); \
    } while (0)
    if (r->prec == SG_FP64)
        SG_RAS_GO(double, r->sinv64.p);
    else if (r->prec == SG_FP32)
        SG_RAS_GO(float, r->sinv32.p);
    else
        SG_RAS_GO(uint16_t, r->sinv16.p);
#undef SG_RAS_GO
#undef SG_RAS_ARGS
#undef SG_RAS_TAIL
    HIP_LAUNCH_OK();
}

namespace {

// Breadth-first levels of the local graph from `start`; unvisited
// components are appended (restarting from their smallest global id).
int bfs_levels(const std::vector<std::vector<int>>& adj, int start,
               const std::vector<int32_t>& gid, std::vector<int>& level_of) {
    const int m = (int)adj.size();
    level_of.assign(m, -1);
    int nlev = 0;
    std::vector<int> frontier{start}, next;
    level_of[start] = 0;
    int visited = 1;
    while (true) {
        while (!frontier.empty()) {
            ++nlev;
            next.clear();
            for (int v : frontier)
                for (int w : adj[v])
                    if (level_of[w] < 0) {
                        level_of[w] = nlev;
                        next.push_back(w);
                        ++visited;
                    }
            frontier.swap(next);
        }
        if (visited == m) break;
        int best = -1;
        for (int v = 0; v < m; ++v)
            if (level_of[v] < 0 && (best < 0 || gid[v] < gid[best])) best = v;
        level_of[best] = nlev;
        frontier.assign(1, best);
        ++visited;
    }
    return nlev;
}

}  // namespace
}  // namespace sg

namespace sg {
namespace {

// Gather the gamma = 0 values of the subdomain matrices from op and factor
// them (block-tridiagonal Schur complements, explicit inverses).
void ras_factor_values(sg_ras* r, const sg_op* op, hipStream_t s) {
    r->op_L = op->L;
    const int64_t mm = (int64_t)r->lent.n;
    if (mm)
        gather_k0_kernel<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>(mm, op->L, r->lent.p,
                                                                       op->vals.p, r->lval.p);
    HIP_LAUNCH_OK();
    const int64_t mc = (int64_t)r->prev_ent.n;
    if (mc) {
        gather_k0_kernel<<<(unsigned)((mc + 255) / 256), 256, 0, s>>>(mc, op->L, r->prev_ent.p,
                                                                       op->vals.p, r->prev_val.p);
        HIP_LAUNCH_OK();
        gather_k0_kernel<<<(unsigned)((mc + 255) / 256), 256, 0, s>>>(mc, op->L, r->next_ent.p,
                                                                       op->vals.p, r->next_val.p);
        HIP_LAUNCH_OK();
    }
    DevBuf<int> d_status(1);
    HIP_OK(hipMemsetAsync(d_status.p, 0, sizeof(int), s));
    const size_t lds = (size_t)2 * kMaxLevel * kMaxLevel * sizeof(double);
    ras_factor_kernel<<<r->n_sub, kRasThreads, lds, s>>>(
        r->sub_node_off.p, r->sub_lev_off.p, r->lev_start.p, r->lev_size.p, r->sinv_off.p,
        r->lrow_ptr.p, r->lcol.p, r->lval.p, r->sinv64.p, r->sinv32.p, r->sinv16.p, (int)r->prec,
        d_status.p);
    HIP_LAUNCH_OK();
    int status = 0;
    d_status.download(&status, 1, s);
    HIP_OK(hipStreamSynchronize(s));
    if (status) SG_THROW(SG_ERR_NUMERIC, "non-positive pivot in a subdomain factorisation");
}

// Explicit inverse rows of the owned nodes of every subdomain: the factored
// sweeps applied to identity blocks of kSetupCols local columns at a time
// (FP64), then narrowed to the storage precision.
constexpr int kSetupCols = 64;

void ras_build_dense(sg_ras* r, hipStream_t s) {
    const int ns = r->n_sub;
    r->Pp = (r->P + 15) / 16 * 16;
    SG_REQUIRE(r->Pp / 16 <= 8, "dense RAS supports P <= 128");
    if (!r->dense_built) {
        r->h_ld.assign(ns, 0);
        r->h_nown.assign(ns, 0);
        r->h_aoff.assign(ns + 1, 0);
        r->h_toff.assign(ns + 1, 0);
        r->h_xoff.assign(ns + 1, 0);
        std::vector<int64_t> own_off(ns + 1, 0);
        std::vector<int32_t> own_pos(r->h_gnode.size(), -1), own_gnode, node_sub;
        std::vector<int32_t> bsub[3], brow[3];
        for (int q = 0; q < ns; ++q) {
            const int a0 = r->h_sub_node_off[q], a1 = r->h_sub_node_off[q + 1];
            int no = 0;
            for (int a = a0; a < a1; ++a) {
                node_sub.push_back(q);
                if (r->h_owned[a]) {
                    own_pos[a] = no++;
                    own_gnode.push_back(r->h_gnode[a]);
                }
            }
            r->h_ld[q] = (a1 - a0 + kDenseLd - 1) / kDenseLd * kDenseLd;
            r->h_nown[q] = no;
            r->h_aoff[q + 1] = r->h_aoff[q] + (int64_t)no * r->h_ld[q];
            r->h_toff[q + 1] = r->h_toff[q] + (int64_t)(no + 63) / 64 * 64 * r->h_ld[q];
            r->h_xoff[q + 1] = r->h_xoff[q] + (int64_t)r->Pp * r->h_ld[q];
            own_off[q + 1] = own_off[q] + no;
            for (int v = 0; v < 3; ++v)
                for (int r0 = 0; r0 < no; r0 += v < 2 ? 4 * kDenseRowChoices[v] : kFusedRows) {
                    bsub[v].push_back(q);
                    brow[v].push_back(r0);
                }
        }
        for (int v = 0; v < 3; ++v) r->nblk[v] = (int)bsub[v].size();
        r->own_pos.upload(own_pos, s);
        r->ld_d.upload(r->h_ld, s);
        r->nown_d.upload(r->h_nown, s);
        r->aoff_d.upload(r->h_aoff, s);
        r->toff_d.upload(r->h_toff, s);
        r->xoff_d.upload(r->h_xoff, s);
        r->own_off_d.upload(own_off, s);
        r->own_gnode.upload(own_gnode, s);
        r->node_sub.upload(node_sub, s);
        for (int v = 0; v < 3; ++v) {
            r->blk_sub[v].upload(bsub[v], s);
            r->blk_row0[v].upload(brow[v], s);
        }
        const size_t ts = r->prec == SG_FP64 ? 8 : (r->prec == SG_FP32 ? 4 : 2);
        int ld_max = 0;
        for (int q = 0; q < ns; ++q) ld_max = std::max(ld_max, r->h_ld[q]);
        int lds_max = 0;
        HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, r->device));
        r->fused_lds = dense_fused_lds(ts, r->Pp, ld_max);
        r->lds_max = (size_t)lds_max;
        r->fused_ok = r->Pp / 16 <= fused_max_nt(r->prec) && r->fused_lds <= (size_t)lds_max;
        r->xg.alloc((size_t)r->h_xoff[ns] * ts);
        HIP_OK(hipMemsetAsync(r->xg.p, 0, r->xg.bytes(), s));
    }
    const int64_t total = r->h_aoff[ns];
    DevBuf<double> rows((size_t)total);
    HIP_OK(hipMemsetAsync(rows.p, 0, (size_t)total * 8, s));
    DevBuf<double> zs_tmp((size_t)r->total_local * kSetupCols);
    int maxn = 0;
    for (int q = 0; q < ns; ++q) maxn = std::max(maxn, r->h_sub_node_off[q + 1] - r->h_sub_node_off[q]);
    const int bmax = r->max_b, nmax = r->max_local;
    const size_t lds = ras_apply_lds(SG_FP64, bmax, kColChunk, nmax, r->max_levels);
    dim3 grid(ns, kSetupCols / kColChunk);
    for (int qb = 0; qb < maxn; qb += kSetupCols) {
#define SG_SETUP_GO(KCP, BM)                                                                       \
    ras_apply_kernel<double, KCP, BM, true><<<grid, kRasThreads, lds, s>>>(                         \
        kSetupCols, kColChunk, bmax, nmax, r->max_levels, r->sub_node_off.p, r->sub_lev_off.p,     \
        r->lev_start.p, r->lev_size.p, r->sinv_off.p, r->sinv64.p, r->gnode.p, r->owned.p,         \
        r->prev_idx.p, r->prev_val.p, r->next_idx.p, r->next_val.p, r->afact.p, nullptr, nullptr,  \
        zs_tmp.p, 1.0, 0.0, qb, r->own_pos.p, r->ld_d.p, r->aoff_d.p, rows.p)
        const bool small = bmax <= 40, narrow = r->max_couple <= 2, wide = r->max_couple > 4;
        if (narrow && small)
            SG_SETUP_GO(2, 40);
        else if (narrow)
            SG_SETUP_GO(2, 64);
        else if (wide)
            SG_SETUP_GO(8, 64);
        else if (small)
            SG_SETUP_GO(4, 40);
        else
            SG_SETUP_GO(4, 64);
#undef SG_SETUP_GO
        HIP_LAUNCH_OK();
    }
    // narrow to the storage precision and rearrange into the tiled order
    const int64_t tiled = r->h_toff[ns];
    int maxo = 0;
    for (int q = 0; q < ns; ++q) maxo = std::max(maxo, r->h_nown[q]);
    const dim3 tg(ns, std::max(1, (maxo + 63) / 64 * kTileBlock));
    // A rebuild (ras_refactor) keeps the buffer when its size is unchanged, so
    // captured Arnoldi-step graphs that read it stay valid.
#define SG_TILE(TS, BUF)                                                                           \
    do {                                                                                           \
        if (BUF.n != (size_t)tiled || !BUF.p) BUF.alloc((size_t)tiled);                            \
        tile_dense_kernel<TS><<<tg, 256, 0, s>>>(r->nown_d.p, r->ld_d.p, r->aoff_d.p, r->toff_d.p, \
                                                 rows.p, BUF.p);                                   \
        HIP_LAUNCH_OK();                                                                           \
    } while (0)
    if (r->prec == SG_FP64)
        SG_TILE(double, r->ainv64);
    else if (r->prec == SG_FP32)
        SG_TILE(float, r->ainv32);
    else
        SG_TILE(uint16_t, r->ainv16);
#undef SG_TILE
    HIP_OK(hipStreamSynchronize(s));
    r->dense_built = true;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int ras_select(sg_ras* r, int dense, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(r != nullptr, "ras is NULL");
        SG_REQUIRE(dense >= 0 && dense <= 3, "path must be 0 (sweep), 1, 2 or 3 (dense)");
        check_device(r->device);
        if (dense && !r->dense_built) ras_build_dense(r, as_stream(stream));
        if (dense == 3 && !r->fused_ok)
            SG_THROW(SG_ERR_UNSUPPORTED, "fused dense RAS needs %zu bytes of LDS and P <= %d",
                     r->fused_lds, 16 * fused_max_nt(r->prec));
        const bool changed = r->use_dense != (dense != 0) || (dense && r->dense_var != dense - 1);
        r->use_dense = dense != 0;
        if (dense) r->dense_var = dense - 1;
        if (changed) graph_cache_purge(r);   // captured steps hold the old path
        return SG_OK;
    });
}

int ras_autotune(sg_ras* r, int reps, double* ms_out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(r != nullptr, "ras is NULL");
        SG_REQUIRE(reps >= 1, "reps must be >= 1");
        check_device(r->device);
        hipStream_t s = as_stream(stream);
        if (!r->dense_built) ras_build_dense(r, s);
        const size_t N = (size_t)r->n * r->P;
        DevBuf<double> R(N), Z(N);
        HIP_OK(hipMemsetAsync(R.p, 0, N * 8, s));
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        // candidates: sweep, dense with 64 and with 32 rows per wave, fused
        // dense (where it fits; -1 otherwise)
        double ms[4] = {0.0, 0.0, 0.0, -1.0};
        try {
            for (int c = 0; c < 4; ++c) {
                if (c == 3 && !r->fused_ok) break;
                r->use_dense = c > 0;
                r->dense_var = c > 0 ? c - 1 : 0;
                ras_apply_ex(r, R.p, Z.p, 1.0, 0.0, s);            // warm-up
                HIP_OK(hipEventRecord(e0, s));
                for (int q = 0; q < reps; ++q) ras_apply_ex(r, R.p, Z.p, 1.0, 0.0, s);
                HIP_OK(hipEventRecord(e1, s));
                HIP_OK(hipEventSynchronize(e1));
                float t = 0.f;
                HIP_OK(hipEventElapsedTime(&t, e0, e1));
                ms[c] = t / reps;
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        int best = 0;
        for (int c = 1; c < 4; ++c)
            if (ms[c] >= 0.0 && ms[c] < ms[best]) best = c;
        r->ms_sweep = ms[0];
        r->ms_dense = std::min(ms[1], ms[2]);
        if (ms[3] >= 0.0) r->ms_dense = std::min(r->ms_dense, ms[3]);
        r->use_dense = best > 0;
        r->dense_var = best > 0 ? best - 1 : 0;
        if (ms_out) for (int c = 0; c < 4; ++c) ms_out[c] = ms[c];
        graph_cache_purge(r);   // captured steps hold the path they were recorded with
        return SG_OK;
    });
}

int ras_path_info(const sg_ras* r, int* dense, int64_t* dense_bytes) {
    return guarded([&]() -> int {
        SG_REQUIRE(r != nullptr, "ras is NULL");
        if (dense) *dense = r->use_dense ? 1 + r->dense_var : 0;
        if (dense_bytes) {
            const int64_t per = r->prec == SG_FP64 ? 8 : (r->prec == SG_FP32 ? 4 : 2);
            *dense_bytes = r->dense_built ? r->h_toff[r->n_sub] * per : 0;
        }
        return SG_OK;
    });
}

int ras_setup(const sg_op* op, const int32_t* owner, int n_sub, int overlap, sg_prec prec,
              sg_ras** out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && owner && out, "null argument");
        SG_REQUIRE(n_sub >= 1 && n_sub <= op->n, "n_sub=%d invalid", n_sub);
        SG_REQUIRE(overlap >= 0 && overlap <= 16, "overlap=%d invalid", overlap);
        SG_REQUIRE(prec == SG_FP64 || prec == SG_FP32 || prec == SG_BF16, "bad precision");
        check_device(op->device);
        hipStream_t s = as_stream(stream);
        const int n = op->n;
        auto r = std::make_unique<sg_ras>();
        r->device = op->device;
        r->n = n; r->P = op->P; r->L = op->L; r->n_sub = n_sub; r->overlap = overlap;
        r->prec = prec;
        r->h_owner.assign(owner, owner + n);
        std::vector<int32_t> cnt(n_sub, 0);
        for (int a = 0; a < n; ++a) {
            SG_REQUIRE(owner[a] >= 0 && owner[a] < n_sub, "owner[%d]=%d out of range", a, owner[a]);
            cnt[owner[a]]++;
        }
        for (int q = 0; q < n_sub; ++q) SG_REQUIRE(cnt[q] > 0, "subdomain %d owns no node", q);
        r->h_own_ptr.assign(n_sub + 1, 0);
        for (int q = 0; q < n_sub; ++q) r->h_own_ptr[q + 1] = r->h_own_ptr[q] + cnt[q];
        r->h_own_nodes.resize(n);
        {
            std::vector<int32_t> fill(r->h_own_ptr.begin(), r->h_own_ptr.end() - 1);
            for (int a = 0; a < n; ++a) r->h_own_nodes[fill[owner[a]]++] = a;
        }

        std::vector<int32_t> sub_node_off(1, 0), sub_lev_off(1, 0), lev_start, lev_size, gnode,
            owned, lrow_ptr(1, 0), lcol, prev_idx, next_idx;
        std::vector<int64_t> lent, sinv_off, prev_ent, next_ent;
        int64_t sinv_count = 0;
        std::vector<int32_t> stamp(n, -1), local_id(n, -1);
        r->h_nlocal.resize(n_sub);
        r->h_nlev.resize(n_sub);
        int max_b = 0;
        for (int sd = 0; sd < n_sub; ++sd) {
            // overlap growth in the mesh graph
            std::vector<int32_t> nodes(r->h_own_nodes.begin() + r->h_own_ptr[sd],
                                       r->h_own_nodes.begin() + r->h_own_ptr[sd + 1]);
            for (int a : nodes) stamp[a] = sd;
            size_t f0 = 0;
            for (int d = 0; d < overlap; ++d) {
                size_t f1 = nodes.size();
                for (size_t q = f0; q < f1; ++q) {
                    int a = nodes[q];
                    for (int64_t e = op->h_graph_ptr[a]; e < op->h_graph_ptr[a + 1]; ++e) {
                        int b = op->h_graph_col[e];
                        if (stamp[b] != sd) { stamp[b] = sd; nodes.push_back(b); }
                    }
                }
                f0 = f1;
            }
            const int m = (int)nodes.size();
            std::sort(nodes.begin(), nodes.end());
            for (int q = 0; q < m; ++q) local_id[nodes[q]] = q;
            // local matrix graph (pattern of K_0 restricted to the subdomain)
            std::vector<std::vector<int>> adj(m);
            for (int q = 0; q < m; ++q) {
                int a = nodes[q];
                for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e) {
                    int b = op->h_col[e];
                    if (b != a && stamp[b] == sd) adj[q].push_back(local_id[b]);
                }
            }
            // pseudo-peripheral start (George-Liu), from the smallest global id
            std::vector<int> lvl;
            int start = 0;
            int ecc = bfs_levels(adj, start, nodes, lvl);
            for (int it = 0; it < 8; ++it) {
                int last = *std::max_element(lvl.begin(), lvl.end());
                int cand = -1;
                for (int q = 0; q < m; ++q)
                    if (lvl[q] == last &&
                        (cand < 0 || adj[q].size() < adj[cand].size() ||
                         (adj[q].size() == adj[cand].size() && nodes[q] < nodes[cand])))
                        cand = q;
                std::vector<int> l2;
                int e2 = bfs_levels(adj, cand, nodes, l2);
                if (e2 <= ecc) break;
                ecc = e2; start = cand; lvl.swap(l2);
            }
            bfs_levels(adj, start, nodes, lvl);
            int nl = *std::max_element(lvl.begin(), lvl.end()) + 1;
            std::vector<int> order(m);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int x, int y) { return lvl[x] < lvl[y]; });
            std::vector<int> pos(m);
            for (int q = 0; q < m; ++q) pos[order[q]] = q;
            // The breadth-first order is a banded ordering: every coupling
            // joins positions at most `band` apart.  Cutting the order into
            // consecutive blocks of `band` nodes therefore also gives a block
            // tridiagonal matrix, with about half as many (wider) blocks as
            // there are level sets -- half the length of the sequential chain
            // of the sweeps.  Used whenever the band fits a block.
            int band = 1;
            for (int qq = 0; qq < m; ++qq)
                for (int w : adj[qq]) band = std::max(band, std::abs(pos[qq] - pos[w]));
            if (band <= kMaxLevel) {
                for (int qq = 0; qq < m; ++qq) lvl[qq] = pos[qq] / band;
                nl = (m + band - 1) / band;
            }
            // levels
            int q = 0;
            std::vector<int> lstart(nl + 1, 0);
            for (int l = 0; l < nl; ++l) {
                int st = q;
                lstart[l] = st;
                while (q < m && lvl[order[q]] == l) ++q;
                int b = q - st;
                if (b > kMaxLevel)
                    SG_THROW(SG_ERR_UNSUPPORTED,
                             "subdomain %d: level set of %d nodes exceeds %d", sd, b, kMaxLevel);
                max_b = std::max(max_b, b);
                lev_start.push_back(st);
                lev_size.push_back(b);
                sinv_off.push_back(sinv_count);
                sinv_count += (int64_t)b * b;
            }
            lstart[nl] = m;
            // local CSR in level order
            for (int qq = 0; qq < m; ++qq) {
                int a = nodes[order[qq]];
                gnode.push_back(a);
                owned.push_back(owner[a] == sd ? 1 : 0);
                std::vector<std::pair<int, int64_t>> ents;
                for (int e = op->h_rowptr[a]; e < op->h_rowptr[a + 1]; ++e) {
                    int b = op->h_col[e];
                    if (stamp[b] == sd) ents.push_back({pos[local_id[b]], (int64_t)e});
                }
                std::sort(ents.begin(), ents.end());
                const int lq = lvl[order[qq]];
                int np = 0, nn = 0;
                size_t base = prev_idx.size();
                prev_idx.resize(base + kCouple, -1);
                next_idx.resize(base + kCouple, -1);
                prev_ent.resize(base + kCouple, -1);
                next_ent.resize(base + kCouple, -1);
                for (auto& pe : ents) {
                    lcol.push_back(pe.first);
                    lent.push_back(pe.second);
                    const int lc = lvl[order[pe.first]];
                    if (lc == lq - 1) {
                        if (np == kCouple)
                            SG_THROW(SG_ERR_UNSUPPORTED, "node couples to more than %d nodes of a level",
                                     kCouple);
                        prev_idx[base + np] = pe.first - lstart[lc];
                        prev_ent[base + np] = pe.second;
                        ++np;
                    } else if (lc == lq + 1) {
                        if (nn == kCouple)
                            SG_THROW(SG_ERR_UNSUPPORTED, "node couples to more than %d nodes of a level",
                                     kCouple);
                        next_idx[base + nn] = pe.first - lstart[lc];
                        next_ent[base + nn] = pe.second;
                        ++nn;
                    } else if (lc != lq) {
                        SG_THROW(SG_ERR_INVALID_ARG, "internal: level structure is not tridiagonal");
                    }
                }
                lrow_ptr.push_back((int32_t)lcol.size());
                r->max_couple = std::max(r->max_couple, std::max(np, nn));
            }
            sub_node_off.push_back((int32_t)gnode.size());
            sub_lev_off.push_back((int32_t)lev_start.size());
            r->h_nlocal[sd] = m;
            if (m > kMaxLocal)
                SG_THROW(SG_ERR_UNSUPPORTED, "subdomain %d has %d nodes (limit %d)", sd, m, kMaxLocal);
            r->max_local = std::max(r->max_local, m);
            r->h_nlev[sd] = nl;
            r->max_levels = std::max(r->max_levels, nl);
            for (int a : nodes) local_id[a] = -1;
        }
        r->total_local = (int64_t)gnode.size();
        r->n_lev = (int64_t)lev_start.size();
        r->sinv_count = sinv_count;
        r->max_b = max_b;
        SG_REQUIRE(lcol.size() < (size_t)INT32_MAX, "local pattern too large");

        r->h_sub_node_off = sub_node_off;
        r->h_gnode = gnode;
        r->h_owned = owned;
        r->sub_node_off.upload(sub_node_off, s);
        r->sub_lev_off.upload(sub_lev_off, s);
        r->lev_start.upload(lev_start, s);
        r->lev_size.upload(lev_size, s);
        r->sinv_off.upload(sinv_off, s);
        r->gnode.upload(gnode, s);
        r->owned.upload(owned, s);
        r->lrow_ptr.upload(lrow_ptr, s);
        r->lcol.upload(lcol, s);
        r->afact.upload(op->h_afact, s);
        r->prev_idx.upload(prev_idx, s);
        r->next_idx.upload(next_idx, s);
        r->lent.upload(lent, s);
        r->prev_ent.upload(prev_ent, s);
        r->next_ent.upload(next_ent, s);
        r->op_nnz = op->nnz;
        r->lval.alloc(lent.size());
        r->prev_val.alloc(prev_ent.size());
        r->next_val.alloc(prev_ent.size());
        r->sinv64.alloc(sinv_count);
        if (prec == SG_FP32) r->sinv32.alloc(sinv_count);
        if (prec == SG_BF16) r->sinv16.alloc(sinv_count);
        r->zs.alloc((size_t)r->total_local * r->P);
        int max_lds = 0;
        HIP_OK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                     op->device));
        const size_t lds = (size_t)2 * kMaxLevel * kMaxLevel * sizeof(double);
        if ((size_t)max_lds < lds)
            SG_THROW(SG_ERR_UNSUPPORTED, "device offers %d bytes of LDS per block, need %zu",
                     max_lds, lds);
        {
            const int nch = (r->P + kColChunk - 1) / kColChunk;
            const int KC = (r->P + nch - 1) / nch;
            size_t need = ras_apply_lds(SG_FP64, max_b, KC, r->max_local, r->max_levels);
            if ((size_t)max_lds < need)
                SG_THROW(SG_ERR_UNSUPPORTED, "RAS apply needs %zu bytes of LDS", need);
        }
        ras_factor_values(r.get(), op, s);
        *out = r.release();
        return SG_OK;
    });
}

// The Kronecker local factor of Ullmann's preconditioner: Gt = sum_i
// (<K_i, K_0>_F / <K_0, K_0>_F) G_i, the G that minimises the Frobenius
// distance of K_0 (x) G to sum_i K_i (x) G_i, and the mixing W = Gt^{-1} G_0
// that turns the mean-based RAS (which divides mode j by <Psi_j^2>) into
// RAS with the local operator K_0 (x) Gt.
void ras_kron_weights(sg_ras* r, const sg_op* op, hipStream_t s) {
    const int L = op->L, P = op->P;
    std::vector<double> v((size_t)op->nnz * L);
    op->vals.download(v.data(), v.size(), s);
    HIP_OK(hipStreamSynchronize(s));
    std::vector<double> t(L, 0.0);
    for (int64_t e = 0; e < op->nnz; ++e) {
        const double k0 = v[(size_t)e * L];
        for (int i = 0; i < L; ++i) t[i] += v[(size_t)e * L + i] * k0;
    }
    if (!(t[0] > 0.0)) SG_THROW(SG_ERR_NUMERIC, "mean stiffness matrix is zero");
    const sg_basis& B = op->basis;
    std::vector<double> G((size_t)P * P, 0.0);
    for (int q = 0; q < B.T; ++q)
        G[(size_t)B.tk[q] * P + B.tj[q]] += (t[B.ti[q]] / t[0]) * B.tv[q];
    r->h_gt = G;
    // Gauss-Jordan with partial pivoting: Ginv = Gt^{-1}
    std::vector<double> A = G, I((size_t)P * P, 0.0);
    for (int k = 0; k < P; ++k) I[(size_t)k * P + k] = 1.0;
    for (int c = 0; c < P; ++c) {
        int piv = c;
        for (int q = c + 1; q < P; ++q)
            if (std::fabs(A[(size_t)q * P + c]) > std::fabs(A[(size_t)piv * P + c])) piv = q;
        if (!(std::fabs(A[(size_t)piv * P + c]) > 0.0))
            SG_THROW(SG_ERR_NUMERIC, "Kronecker factor Gt is singular");
        if (piv != c)
            for (int q = 0; q < P; ++q) {
                std::swap(A[(size_t)piv * P + q], A[(size_t)c * P + q]);
                std::swap(I[(size_t)piv * P + q], I[(size_t)c * P + q]);
            }
        const double d = 1.0 / A[(size_t)c * P + c];
        for (int q = 0; q < P; ++q) {
            A[(size_t)c * P + q] *= d;
            I[(size_t)c * P + q] *= d;
        }
        for (int q2 = 0; q2 < P; ++q2) {
            if (q2 == c) continue;
            const double f = A[(size_t)q2 * P + c];
            if (f == 0.0) continue;
            for (int q = 0; q < P; ++q) {
                A[(size_t)q2 * P + q] -= f * A[(size_t)c * P + q];
                I[(size_t)q2 * P + q] -= f * I[(size_t)c * P + q];
            }
        }
    }
    const int Pw = kron_wcols(P);                // columns padded with zeros
    std::vector<double> W((size_t)P * Pw, 0.0);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j) W[(size_t)k * Pw + j] = I[(size_t)k * P + j] * op->h_afact[j];
    r->kron_w.upload(W, s);
    // Gt^{-1} [P x Pp] for the output mixing of the fused path
    const int Pp = 16 * ((P + 15) / 16);
    std::vector<double> post((size_t)P * Pp, 0.0);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j) post[(size_t)k * Pp + j] = I[(size_t)k * P + j];
    r->kron_post.upload(post, s);
    int lds_max = 0;
    HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, r->device));
    r->post_pp = Pp;
    r->post_lds = dense_post_lds(P, Pp, r->prec == SG_FP64 ? 8 : 4);
    r->post_ok = r->post_lds <= (size_t)lds_max;
    const size_t N = (size_t)r->n * P;
    if (r->kron_t.n < N) r->kron_t.alloc(N);
    HIP_OK(hipStreamSynchronize(s));
}

int ras_set_local(sg_ras* r, const sg_op* op, sg_local_kind mode, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(r && op, "null argument");
        SG_REQUIRE(mode == SG_LOCAL_MEAN || mode == SG_LOCAL_KRON, "bad local-solve kind %d",
                   (int)mode);
        check_device(op->device);
        SG_REQUIRE(op->device == r->device, "ras and op on different devices");
        SG_REQUIRE(op->n == r->n && op->nnz == r->op_nnz && op->P == r->P,
                   "op does not have the pattern the ras was built for");
        if (mode == SG_LOCAL_KRON) ras_kron_weights(r, op, as_stream(stream));
        if (r->local_mode != mode) sg::graph_cache_purge(r);   // captured steps hold the old mode
        r->local_mode = mode;
        return SG_OK;
    });
}

int ras_local_factor(const sg_ras* r, double* gt) {
    return guarded([&]() -> int {
        SG_REQUIRE(r && gt, "null argument");
        SG_REQUIRE(r->local_mode == SG_LOCAL_KRON, "local solves are not Kronecker");
        std::copy(r->h_gt.begin(), r->h_gt.end(), gt);
        return SG_OK;
    });
}

int ras_refactor(sg_ras* r, const sg_op* op, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(r && op, "null argument");
        check_device(op->device);
        SG_REQUIRE(op->device == r->device, "ras and op on different devices");
        SG_REQUIRE(op->n == r->n && op->nnz == r->op_nnz && op->P == r->P,
                   "op does not have the pattern the ras was built for");
        const void* before[3] = {r->ainv64.p, r->ainv32.p, r->ainv16.p};
        ras_factor_values(r, op, as_stream(stream));
        if (r->dense_built) ras_build_dense(r, as_stream(stream));
        if (r->local_mode == SG_LOCAL_KRON) ras_kron_weights(r, op, as_stream(stream));
        // graphs captured earlier hold the dense rows' address: drop them if it moved
        if (before[0] != r->ainv64.p || before[1] != r->ainv32.p || before[2] != r->ainv16.p)
            sg::graph_cache_purge(r);
        return SG_OK;
    });
}

int ras_info(const sg_ras* r, int32_t* n_local, int32_t* n_levels, int64_t* factor_bytes) {
    return guarded([&]() -> int {
        SG_REQUIRE(r != nullptr, "ras is NULL");
        if (n_local) std::memcpy(n_local, r->h_nlocal.data(), r->n_sub * sizeof(int32_t));
        if (n_levels) std::memcpy(n_levels, r->h_nlev.data(), r->n_sub * sizeof(int32_t));
        if (factor_bytes) {
            int64_t per = r->prec == SG_FP64 ? 8 : (r->prec == SG_FP32 ? 4 : 2);
            *factor_bytes = r->sinv_count * per;
        }
        return SG_OK;
    });
}

int ras_apply(const sg_ras* r, const double* R, double* Z, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(r && R && Z, "null argument");
        SG_REQUIRE(R != Z, "R and Z must not alias");
        check_device(r->device);
        ras_apply_ex(r, R, Z, 1.0, 0.0, as_stream(stream));
        return SG_OK;
    });
}

void sg_destroy_ras(sg_ras* r) {
    sg::graph_cache_purge(r);
    delete r;
}

}  // extern "C"

namespace sg {
const std::vector<int32_t>& ras_owner(const sg_ras* r) { return r->h_owner; }
int ras_nsub(const sg_ras* r) { return r->n_sub; }
int ras_device(const sg_ras* r) { return r->device; }
int ras_n(const sg_ras* r) { return r->n; }
}  // namespace sg
