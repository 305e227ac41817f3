// Nonlinear stochastic Galerkin problem and Newton's method.
//
// The paper's nonlinear model (Eq. NLP_StrongPDE) is -div(c(x,xi) q(u)
// grad u) = f with a polynomial q, Galerkin-projected and linearised by
// Picard iterations (Eqs. stonlp_system, vectorvalPDENL).  Here
// q(u) = kappa(u) = 1 + a1 u + a2 u^2 (the paper's 1 + alpha u is a1 = alpha,
// a2 = 0), f = 1, homogeneous Dirichlet data, and the Galerkin system
// R(U) = F e_0 - A(U) = 0 is solved by inexact Newton with backtracking or by
// the paper's Picard iteration U <- U + K1(U)^{-1} R(U) = K1(U)^{-1} F e_0,
// each linear system by FGMRES with the two-grid RAS cycle.
//
// Exact Galerkin integrals without quadrature.  With P1 elements and the
// centroid value u_T = (u_1 + u_2 + u_3)/3 in kappa,
//   A(U)[a, m]          = sum_T |T| E[c_T kappa(u_T) (grad u_T . grad phi_a) Psi_m]
//   dA/dU[(a,m),(b,n)]  = sum_T |T| ( E[c_T kappa(u_T) Psi_m Psi_n] grad phi_a . grad phi_b
//                                   + E[c_T kappa'(u_T) (grad u_T . grad phi_a) Psi_m Psi_n] / 3 ).
// Both only need the chaos coefficients of degree <= 2p of the element
// fields  w_T = c_T kappa(u_T)  and  y_{T,a} = c_T kappa'(u_T) (grad u_T . grad phi_a),
// since Psi_m Psi_n has degree <= 2p.  Those follow exactly from products of
// chaos expansions (u_T^2 and u_T * flux have degree 2p; the product with
// the degree-p_in coefficient c_T is projected onto degree <= 2p):
//   (f g)_gamma = sum_{i,j} f_i g_j <Psi_i Psi_j Psi_gamma> / gamma!.
// Summing element contributions gives the Jacobian in the same
// Kronecker-sum form as the linear operator, with L2 = C(M+2p, 2p) input
// terms:  J = sum_gamma (K1_gamma + K2_gamma) (x) T_gamma,  T_gamma[n][m] =
// <Psi_gamma Psi_n Psi_m>, and A(U) = (sum_gamma K1_gamma (x) T_gamma) U.
// K1_0 is the stiffness matrix of the mean coefficient E[c kappa(u_T)], the
// operator of the mean-based RAS local solves.
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

struct sg_nl {
    int device = 0;
    int n = 0, P = 0, M = 0, p = 0, L_in = 0, L2 = 0, n_tri = 0;
    double a1 = 0.0, a2 = 0.5;
    std::unique_ptr<sg_op> j1, jac;          // K1 (residual, RAS) and K1 + K2 (Jacobian)
    sg::DevBuf<int32_t> edof;                // [n_tri][3]
    sg::ElementData ed;
    sg::DevBuf<int64_t> cptr;
    sg::DevBuf<int32_t> cref;
    // chaos product tables, both sorted by the output term gamma
    sg::DevBuf<int32_t> sq_ptr, sq_ij;       // (i < P, j < P) -> gamma < L2, packed i | j << 16
    sg::DevBuf<double> sq_v;
    sg::DevBuf<int32_t> cm_ptr, cm_kd;       // (k < L_in, d < L2) -> gamma < L2
    sg::DevBuf<double> cm_v;
    sg::DevBuf<double> inv_gfact;            // 1 / gamma!
    sg::DevBuf<double> w1, yt;               // [n_tri][L2], [n_tri][3][L2]
    sg::DevBuf<double> B;                    // F e_0, [n][P]
    sg::DevBuf<int32_t> mode_deg;            // total degree of each chaos mode [P]
    sg_basis basis;                          // the basis of u and c
    std::vector<double> h_xy;                // mesh (for new coefficient fields)
    std::vector<int32_t> h_tri;
    int n_vert = 0;
};

namespace sg {
namespace {

constexpr int kWaves = 4;
constexpr int kGuessSweeps = 3;       // Jacobi sweeps smoothing a predicted guess
constexpr double kGuessOmega = 0.6;   // their damping

__device__ __forceinline__ void wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// One wave per element: chaos coefficients (degree <= 2p) of w_T and of
// y_{T,a} |T| / 3 (the factor 1/3 of d u_T / d u_b folded in).
__global__ __launch_bounds__(64 * kWaves) void nl_element_kernel(
    int n_tri, int P, int L_in, int L2, double a1, double a2, const int32_t* __restrict__ edof,
    const double* __restrict__ ek, const double* __restrict__ ec, const double* __restrict__ U,
    const int32_t* __restrict__ sq_ptr, const int32_t* __restrict__ sq_ij,
    const double* __restrict__ sq_v, const int32_t* __restrict__ cm_ptr,
    const int32_t* __restrict__ cm_kd, const double* __restrict__ cm_v,
    const double* __restrict__ inv_gfact, double* __restrict__ w1, double* __restrict__ yt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t per_wave = (size_t)7 * P + L_in + 4 * (size_t)L2;
    double* ub = reinterpret_cast<double*>(smem_raw) + wave * per_wave;   // [3][P]
    double* uT = ub + 3 * P;                                               // [P]
    double* fl = uT + P;                                                   // [3][P]  |T| flux
    double* c = fl + 3 * P;                                                // [L_in]
    double* kap = c + L_in;                                                // [L2]
    double* v = kap + L2;                                                  // [3][L2]
    for (int t = blockIdx.x * kWaves + wave; t < n_tri; t += gridDim.x * kWaves) {
        const double* e9 = ek + (size_t)t * 9;
        for (int q = lane; q < 3 * P; q += 64) {
            const int b = q / P, j = q - (q / P) * P;
            const int d = edof[3 * t + b];
            ub[q] = d >= 0 ? U[(size_t)d * P + j] : 0.0;
        }
        for (int q = lane; q < L_in; q += 64) c[q] = ec[(size_t)t * L_in + q];
        wave_sync();
        for (int j = lane; j < P; j += 64) {
            const double u0 = ub[j], u1 = ub[P + j], u2 = ub[2 * P + j];
            uT[j] = (u0 + u1 + u2) / 3.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                fl[a * P + j] = e9[3 * a] * u0 + e9[3 * a + 1] * u1 + e9[3 * a + 2] * u2;
        }
        wave_sync();
        // kappa(u_T) = 1 + a1 u_T + a2 u_T^2 and kappa'(u_T) flux_a =
        // a1 flux_a + 2 a2 u_T flux_a, of degree <= 2p (the first P terms of the
        // degree-2p basis are the degree-p basis in the same order)
        for (int g = lane; g < L2; g += 64) {
            double s = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
            for (int q = sq_ptr[g]; q < sq_ptr[g + 1]; ++q) {
                const int ij = sq_ij[q];
                const int i = ij & 0xffff, j = ij >> 16;
                const double mu = sq_v[q] * uT[i];
                s = fma(mu, uT[j], s);
                v0 = fma(mu, fl[j], v0);
                v1 = fma(mu, fl[P + j], v1);
                v2 = fma(mu, fl[2 * P + j], v2);
            }
            const double ig = inv_gfact[g];
            const bool lin = g < P;
            kap[g] = (g == 0 ? 1.0 : 0.0) + (lin ? a1 * uT[g] : 0.0) + a2 * s * ig;
            v[g] = (lin ? a1 * fl[g] : 0.0) + 2.0 * a2 * v0 * ig;
            v[L2 + g] = (lin ? a1 * fl[P + g] : 0.0) + 2.0 * a2 * v1 * ig;
            v[2 * L2 + g] = (lin ? a1 * fl[2 * P + g] : 0.0) + 2.0 * a2 * v2 * ig;
        }
        wave_sync();
        // products with c_T, projected onto degree <= 2p
        const double yscale = 1.0 / 3.0;
        for (int g = lane; g < L2; g += 64) {
            double w = 0.0, y0 = 0.0, y1 = 0.0, y2 = 0.0;
            for (int q = cm_ptr[g]; q < cm_ptr[g + 1]; ++q) {
                const int kd = cm_kd[q];
                const int k = kd & 0xffff, d = kd >> 16;
                const double mc = cm_v[q] * c[k];
                w = fma(mc, kap[d], w);
                y0 = fma(mc, v[d], y0);
                y1 = fma(mc, v[L2 + d], y1);
                y2 = fma(mc, v[2 * L2 + d], y2);
            }
            const double ig = inv_gfact[g];
            w1[(size_t)t * L2 + g] = w * ig;
            yt[((size_t)t * 3 + 0) * L2 + g] = yscale * y0 * ig;
            yt[((size_t)t * 3 + 1) * L2 + g] = yscale * y1 * ig;
            yt[((size_t)t * 3 + 2) * L2 + g] = yscale * y2 * ig;
        }
        wave_sync();
    }
}

// One thread per (entry, gamma): fixed-order sum of element contributions.
__global__ void nl_entry_kernel(int64_t nnz, int L2, const int64_t* __restrict__ cptr,
                                const int32_t* __restrict__ cref, const double* __restrict__ ek,
                                const double* __restrict__ w1, const double* __restrict__ yt,
                                double* __restrict__ k1, double* __restrict__ jv) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nnz * L2) return;
    const int64_t e = idx / L2;
    const int g = (int)(idx - e * L2);
    double a1 = 0.0, a2 = 0.0;
    for (int64_t q = cptr[e]; q < cptr[e + 1]; ++q) {
        const int32_t r = cref[q];
        const int32_t t = r / 9, pr = r - 9 * (r / 9), la = pr / 3;
        a1 = fma(w1[(size_t)t * L2 + g], ek[(size_t)t * 9 + pr], a1);
        a2 += yt[((size_t)t * 3 + la) * L2 + g];
    }
    k1[idx] = a1;
    jv[idx] = a1 + a2;
}

__global__ void nl_rhs_kernel(int n, int P, const double* __restrict__ F, double* __restrict__ B) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * P) return;
    const int64_t a = idx / P;
    B[idx] = (idx - a * P == 0) ? F[a] : 0.0;
}

// Y = X + lam * D
__global__ void nl_axpy_kernel(int64_t N, double lam, const double* __restrict__ X,
                               const double* __restrict__ D, double* __restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < N) Y[idx] = fma(lam, D[idx], X[idx]);
}

__global__ void nl_fill_kernel(int64_t N, double v, double* __restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < N) Y[idx] = v;
}

// Y[a, k] = X[a, k] if mode k has total degree d, else 0.
__global__ void nl_degree_part_kernel(int64_t N, int P, int d, const int32_t* __restrict__ deg,
                                      const double* __restrict__ X, double* __restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int k = (int)(idx % P);
    Y[idx] = deg[k] == d ? X[idx] : 0.0;
}

// One damped Jacobi sweep with the mean-coefficient diagonal:
// X[a, k] += omega R[a, k] / (K1_0[a, a] k!).
__global__ void nl_jacobi_kernel(int n, int P, int L2, const int32_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ col, const double* __restrict__ k1,
                                 const double* __restrict__ afact, double omega,
                                 const double* __restrict__ R, double* __restrict__ X) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * P) return;
    const int a = (int)(idx / P), k = (int)(idx - (int64_t)a * P);
    double d = 0.0;
    for (int e = rowptr[a]; e < rowptr[a + 1]; ++e)
        if (col[e] == a) d = k1[(size_t)e * L2];
    if (d > 0.0) X[idx] += omega * R[idx] / (d * afact[k]);
}

// Y = X + sum_d beta_d W_d, W_d the degree-d part of X (beta on the device).
__global__ void nl_degree_scale_kernel(int64_t N, int P, const int32_t* __restrict__ deg,
                                       const double* __restrict__ beta, const double* __restrict__ X,
                                       double* __restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int k = (int)(idx % P);
    Y[idx] = X[idx] * (1.0 + beta[deg[k]]);
}

inline unsigned grid1d(int64_t N) { return (unsigned)((N + 255) / 256); }

// Operators sharing the unpruned P1 pattern: the off-diagonal Jacobian
// entries of an element are non-zero even where grad phi_a . grad phi_b = 0.
std::unique_ptr<sg_op> make_op(const MeshPattern& mp, int n, const sg_basis& jb, hipStream_t s) {
    auto op = std::make_unique<sg_op>();
    op->device = current_device();
    op->n = n; op->P = jb.P; op->L = jb.L; op->M = jb.M;
    op->nnz = (int64_t)mp.col.size();
    op->max_row = mp.max_row;
    op->basis = jb;
    op->h_afact = jb.afact;
    op->h_rowptr = mp.rowptr;
    op->h_col = mp.col;
    op->h_graph_ptr = mp.graph_ptr;
    op->h_graph_col = mp.graph_col;
    op->rowptr.upload(mp.rowptr, s);
    op->col.upload(mp.col, s);
    op->vals.alloc((size_t)op->nnz * jb.L);
    op->F.alloc(n);
    op->afact.upload(jb.afact, s);
    upload_triples(jb, op->tr, s);
    build_row_tiled(op.get(), s);      // wide bases (L2 > 32): the row-tiled matvec
    return op;
}

// Assemble K1 and J at U and form R = F e_0 - A(U) (R may be null).
void nl_eval(sg_nl* nl, const double* U, double* R, hipStream_t s) {
    const size_t per_wave = ((size_t)7 * nl->P + nl->L_in + 4 * (size_t)nl->L2) * 8;
    const unsigned blocks = (unsigned)std::min<int64_t>((nl->n_tri + kWaves - 1) / kWaves, 16384);
    nl_element_kernel<<<blocks, 64 * kWaves, per_wave * kWaves, s>>>(
        nl->n_tri, nl->P, nl->L_in, nl->L2, nl->a1, nl->a2, nl->edof.p, nl->ed.ek.p, nl->ed.ec.p, U,
        nl->sq_ptr.p, nl->sq_ij.p, nl->sq_v.p, nl->cm_ptr.p, nl->cm_kd.p, nl->cm_v.p,
        nl->inv_gfact.p, nl->w1.p, nl->yt.p);
    HIP_LAUNCH_OK();
    const int64_t work = nl->jac->nnz * nl->L2;
    nl_entry_kernel<<<grid1d(work), 256, 0, s>>>(nl->jac->nnz, nl->L2, nl->cptr.p, nl->cref.p,
                                                 nl->ed.ek.p, nl->w1.p, nl->yt.p, nl->j1->vals.p,
                                                 nl->jac->vals.p);
    HIP_LAUNCH_OK();
    refresh_row_tiled(nl->j1.get(), s);
    refresh_row_tiled(nl->jac.get(), s);
    if (R) kron_matvec(nl->j1->csr(), nl->L2, nl->j1->tr, U, R, -1.0, 1.0, nl->B.p, s);
}

struct RasDel {
    void operator()(sg_ras* r) const { if (r) sg_destroy_ras(r); }
};
struct AmgDel {
    void operator()(sg_amg* a) const { if (a) sg_destroy_amg(a); }
};

inline void check_status(int st, const char* what) {
    if (st < 0) SG_THROW(st, "%s: %s", what, sg_last_error());
}

// R, D, U_trial, R_trial, partial sums, scalars, then the Krylov workspace.
size_t newton_ws(int n, int P, int n_sub, sg_coarse_kind coarse, int restart) {
    const size_t N = (size_t)n * P;
    const int ns = coarse == SG_COARSE_NONE ? -1 : n_sub;
    return 4 * align_up(N * 8) + align_up(kMaxRedBlocks * 8) + 256 + fgmres_ws_ns(n, P, ns, restart);
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int sg_nl_setup(const sg_basis* b, int n_vert, const double* xy, int n_tri, const int32_t* tri,
                const int32_t* dof, int n, const double* g0, const double* g, double a1, double a2,
                sg_nl** out, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(b && out, "null argument");
        SG_REQUIRE(std::isfinite(a1), "a1 must be finite");
        SG_REQUIRE(std::isfinite(a2) && a2 >= 0.0, "a2 must be finite and >= 0");
        hipStream_t s = as_stream(stream);
        validate_mesh(n_vert, xy, n_tri, tri, dof, n);
        auto nl = std::make_unique<sg_nl>();
        nl->device = current_device();
        nl->n = n; nl->P = b->P; nl->M = b->M; nl->p = b->p; nl->L_in = b->L; nl->n_tri = n_tri;
        nl->a1 = a1;
        nl->a2 = a2;
        const int deg2 = 2 * b->p;
        nl->L2 = b->M == 0 ? 1 : binom(b->M + deg2, deg2);
        SG_REQUIRE(nl->L2 < 65536, "2p-degree basis too large (%d terms)", nl->L2);

        // Jacobian basis: input terms of degree <= 2p, modes of degree <= p
        sg_basis jb;
        jb.M = b->M; jb.p_in = deg2; jb.p = b->p; jb.P = b->P; jb.L = nl->L2;
        jb.alpha = b->alpha;
        jb.afact = b->afact;
        {
            SparseTriples st;
            sparse_triples(b->M, deg2, nl->L2, b->P, b->P, st);
            jb.ti = std::move(st.a); jb.tj = std::move(st.b); jb.tk = std::move(st.c);
            jb.tv = std::move(st.v);
            jb.T = (int)jb.tv.size();
        }
        // product tables
        std::vector<int32_t> alpha2;
        int cnt = 0;
        enumerate(b->M, deg2, alpha2, cnt);
        std::vector<double> igf(nl->L2, 1.0);
        for (int q = 0; q < nl->L2; ++q) {
            double f = 1.0;
            for (int d = 0; d < b->M; ++d)
                for (int v = 2; v <= alpha2[(size_t)q * b->M + d]; ++v) f *= v;
            igf[q] = 1.0 / f;
        }
        auto pack_by_c = [&](const SparseTriples& st, int nc, DevBuf<int32_t>& ptr,
                             DevBuf<int32_t>& ab, DevBuf<double>& val) {
            std::vector<int32_t> hp(nc + 1, 0), hab(st.v.size());
            for (size_t q = 0; q < st.v.size(); ++q) {
                hp[st.c[q] + 1]++;
                hab[q] = st.a[q] | (st.b[q] << 16);
            }
            for (int q = 0; q < nc; ++q) hp[q + 1] += hp[q];
            ptr.upload(hp, s);
            ab.upload(hab, s);
            val.upload(st.v, s);
        };
        {
            SparseTriples sq, cm;
            sparse_triples(b->M, deg2, b->P, b->P, nl->L2, sq);
            sparse_triples(b->M, deg2, b->L, nl->L2, nl->L2, cm);
            pack_by_c(sq, nl->L2, nl->sq_ptr, nl->sq_ij, nl->sq_v);
            pack_by_c(cm, nl->L2, nl->cm_ptr, nl->cm_kd, nl->cm_v);
        }
        nl->inv_gfact.upload(igf, s);

        // mesh: unpruned pattern, contributions, element data
        MeshPattern mp;
        mesh_pattern(n_vert, xy, n_tri, tri, dof, n, false, mp);
        element_data(*b, n_vert, xy, n_tri, tri, g0, g, nl->ed, s);
        std::vector<int32_t> ed3((size_t)n_tri * 3);
        for (size_t q = 0; q < ed3.size(); ++q) ed3[q] = dof[tri[q]];
        nl->edof.upload(ed3, s);
        nl->cptr.upload(mp.cptr, s);
        nl->cref.upload(mp.cref, s);
        nl->j1 = make_op(mp, n, jb, s);
        nl->jac = make_op(mp, n, jb, s);
        load_vector(n, nl->j1->rowptr.p, nl->j1->col.p, nl->cptr.p, nl->cref.p, nl->ed.earea.p,
                    nl->j1->F.p, s);
        HIP_OK(hipMemcpyAsync(nl->jac->F.p, nl->j1->F.p, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        nl->B.alloc((size_t)n * b->P);
        nl_rhs_kernel<<<grid1d((int64_t)n * b->P), 256, 0, s>>>(n, b->P, nl->j1->F.p, nl->B.p);
        HIP_LAUNCH_OK();
        nl->w1.alloc((size_t)n_tri * nl->L2);
        nl->yt.alloc((size_t)n_tri * 3 * nl->L2);
        std::vector<int32_t> deg(b->P, 0);
        for (int k = 0; k < b->P; ++k)
            for (int d = 0; d < b->M; ++d) deg[k] += b->alpha[(size_t)k * b->M + d];
        nl->mode_deg.upload(deg, s);
        nl->basis = *b;
        nl->n_vert = n_vert;
        nl->h_xy.assign(xy, xy + (size_t)n_vert * 2);
        nl->h_tri.assign(tri, tri + (size_t)n_tri * 3);
        HIP_OK(hipStreamSynchronize(s));
        *out = nl.release();
        return SG_OK;
    });
}

int sg_nl_set_coefficients(sg_nl* nl, const double* g0, const double* g, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl != nullptr, "nl is NULL");
        check_device(nl->device);
        hipStream_t s = as_stream(stream);
        element_data(nl->basis, nl->n_vert, nl->h_xy.data(), nl->n_tri, nl->h_tri.data(), g0, g,
                     nl->ed, s);
        HIP_OK(hipStreamSynchronize(s));
        return SG_OK;
    });
}

size_t newton_guess_workspace_bytes(const sg_nl* nl) {
    if (!nl) return 0;
    const size_t vb = align_up((size_t)nl->n * nl->P * 8);
    return (size_t)(2 * (nl->p + 1) + 2) * vb + align_up(kMaxRedBlocks * 8) + 512;
}

int newton_guess(sg_nl* nl, const double* U_pred, double* U0, double* relres, int* choice,
                 void* ws, size_t ws_bytes, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl && U_pred && U0, "null argument");
        SG_REQUIRE(U_pred != U0, "U_pred and U0 must not alias");
        check_device(nl->device);
        const size_t need = newton_guess_workspace_bytes(nl);
        if (!ws || ws_bytes < need)
            SG_THROW(SG_ERR_WORKSPACE, "guess workspace too small (%zu < %zu)", ws_bytes, need);
        hipStream_t s = as_stream(stream);
        const int D = nl->p + 1;
        const int64_t N = (int64_t)nl->n * nl->P;
        const size_t vb = align_up((size_t)N * 8);
        char* p = reinterpret_cast<char*>(ws);
        double* R = reinterpret_cast<double*>(p);
        double* T = reinterpret_cast<double*>(p + vb);
        auto Wd = [&](int d) { return reinterpret_cast<double*>(p + (2 + d) * vb); };
        auto JWd = [&](int d) { return reinterpret_cast<double*>(p + (2 + D + d) * vb); };
        double* part = reinterpret_cast<double*>(p + (2 + 2 * D) * vb);
        double* scal = reinterpret_cast<double*>(p + (2 + 2 * D) * vb + align_up(kMaxRedBlocks * 8));
        double* beta_d = scal + 8;
        const double fn = std::sqrt(host_dot(N, nl->B.p, nl->B.p, part, scal, s));
        SG_REQUIRE(fn > 0.0, "the forcing is zero");
        // residual at the prediction
        nl_eval(nl, U_pred, R, s);
        const double r_pred = std::sqrt(host_dot(N, R, R, part, scal, s));
        // smoothing: damped Jacobi sweeps remove the rough part of the error,
        // to which the residual is most sensitive
        double* S = Wd(0);
        HIP_OK(hipMemcpyAsync(S, U_pred, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
        for (int sweep = 0; sweep < kGuessSweeps; ++sweep) {
            nl_jacobi_kernel<<<grid1d(N), 256, 0, s>>>(nl->n, nl->P, nl->L2, nl->j1->rowptr.p,
                                                       nl->j1->col.p, nl->j1->vals.p, nl->j1->afact.p,
                                                       kGuessOmega, R, S);
            HIP_LAUNCH_OK();
            nl_eval(nl, S, R, s);
        }
        const double r_smooth = std::sqrt(host_dot(N, R, R, part, scal, s));
        HIP_OK(hipMemcpyAsync(T, S, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
        HIP_OK(hipMemcpyAsync(U0, S, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
        // Gauss-Newton step restricted to the degree parts of the smoothed field
        std::vector<double> G((size_t)D * D, 0.0), h(D, 0.0), beta(D, 0.0);
        for (int d = 0; d < D; ++d) {
            nl_degree_part_kernel<<<grid1d(N), 256, 0, s>>>(N, nl->P, d, nl->mode_deg.p, T, Wd(d));
            HIP_LAUNCH_OK();
            kron_matvec(nl->jac->csr(), nl->L2, nl->jac->tr, Wd(d), JWd(d), 1.0, 0.0, nullptr, s);
        }
        for (int d = 0; d < D; ++d) {
            h[d] = host_dot(N, JWd(d), R, part, scal, s);
            for (int e = 0; e <= d; ++e)
                G[(size_t)d * D + e] = G[(size_t)e * D + d] = host_dot(N, JWd(d), JWd(e), part, scal, s);
        }
        // Cholesky of the small Gram matrix; degree parts that vanish are skipped
        std::vector<int> act;
        for (int d = 0; d < D; ++d)
            if (G[(size_t)d * D + d] > 0.0) act.push_back(d);
        const int na = (int)act.size();
        std::vector<double> A((size_t)na * na), y(na);
        for (int i = 0; i < na; ++i) {
            y[i] = h[act[i]];
            for (int j = 0; j < na; ++j) A[(size_t)i * na + j] = G[(size_t)act[i] * D + act[j]];
        }
        bool ok = true;
        for (int j = 0; j < na && ok; ++j) {
            double dj = A[(size_t)j * na + j];
            for (int k = 0; k < j; ++k) dj -= A[(size_t)j * na + k] * A[(size_t)j * na + k];
            if (!(dj > 1e-14 * A[(size_t)j * na + j])) { ok = false; break; }
            dj = std::sqrt(dj);
            A[(size_t)j * na + j] = dj;
            for (int i = j + 1; i < na; ++i) {
                double v = A[(size_t)i * na + j];
                for (int k = 0; k < j; ++k) v -= A[(size_t)i * na + k] * A[(size_t)j * na + k];
                A[(size_t)i * na + j] = v / dj;
            }
        }
        if (ok) {
            for (int i = 0; i < na; ++i) {
                double v = y[i];
                for (int k = 0; k < i; ++k) v -= A[(size_t)i * na + k] * y[k];
                y[i] = v / A[(size_t)i * na + i];
            }
            for (int i = na - 1; i >= 0; --i) {
                double v = y[i];
                for (int k = i + 1; k < na; ++k) v -= A[(size_t)k * na + i] * y[k];
                y[i] = v / A[(size_t)i * na + i];
            }
            for (int i = 0; i < na; ++i) beta[act[i]] = y[i];
        }
        HIP_OK(hipMemcpyAsync(beta_d, beta.data(), D * sizeof(double), hipMemcpyHostToDevice, s));
        double r_proj = NAN;
        if (ok) {
            nl_degree_scale_kernel<<<grid1d(N), 256, 0, s>>>(N, nl->P, nl->mode_deg.p, beta_d, T, T);
            HIP_LAUNCH_OK();
            nl_eval(nl, T, R, s);
            r_proj = std::sqrt(host_dot(N, R, R, part, scal, s));
        }
        // U0 holds the smoothed field; the projected one replaces it if better
        double r_sm = r_smooth;
        if (ok && std::isfinite(r_proj) && r_proj < r_sm) {
            HIP_OK(hipMemcpyAsync(U0, T, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
            r_sm = r_proj;
        }
        // the candidate with the smallest residual; the zero guess has ||R|| = ||F||
        int c = 0;
        double best = fn;
        if (std::isfinite(r_pred) && r_pred < best) { c = 1; best = r_pred; }
        if (std::isfinite(r_sm) && r_sm < best) { c = 2; best = r_sm; }
        if (c == 0) {
            nl_fill_kernel<<<grid1d(N), 256, 0, s>>>(N, 0.0, U0);
            HIP_LAUNCH_OK();
        } else if (c == 1) {
            HIP_OK(hipMemcpyAsync(U0, U_pred, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
        }
        HIP_OK(hipStreamSynchronize(s));
        if (relres) {
            relres[0] = 1.0;
            relres[1] = r_pred / fn;
            relres[2] = r_sm / fn;
        }
        if (choice) *choice = c;
        return SG_OK;
    });
}

int sg_nl_info(const sg_nl* nl, int* n, int* P, int* L2, int64_t* nnz) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl != nullptr, "nl is NULL");
        if (n) *n = nl->n;
        if (P) *P = nl->P;
        if (L2) *L2 = nl->L2;
        if (nnz) *nnz = nl->jac->nnz;
        return SG_OK;
    });
}

int sg_nl_eval(sg_nl* nl, const double* U, double* R, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl && U, "null argument");
        SG_REQUIRE(U != R, "U and R must not alias");
        check_device(nl->device);
        nl_eval(nl, U, R, as_stream(stream));
        return SG_OK;
    });
}

int sg_nl_jac_apply(const sg_nl* nl, const double* X, double* Y, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl && X && Y, "null argument");
        SG_REQUIRE(X != Y, "X and Y must not alias");
        check_device(nl->device);
        kron_matvec(nl->jac->csr(), nl->L2, nl->jac->tr, X, Y, 1.0, 0.0, nullptr,
                    as_stream(stream));
        return SG_OK;
    });
}

int sg_nl_export(const sg_nl* nl, int64_t* rowptr, int32_t* col, double* k1, double* jac) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl != nullptr, "nl is NULL");
        check_device(nl->device);
        const sg_op* op = nl->jac.get();
        if (rowptr)
            for (int a = 0; a <= op->n; ++a) rowptr[a] = op->h_rowptr[a];
        if (col) std::memcpy(col, op->h_col.data(), op->nnz * sizeof(int32_t));
        if (k1) nl->j1->vals.download(k1, (size_t)op->nnz * nl->L2, nullptr);
        if (jac) op->vals.download(jac, (size_t)op->nnz * nl->L2, nullptr);
        HIP_OK(hipDeviceSynchronize());
        return SG_OK;
    });
}

const sg_op* sg_nl_mean_op(const sg_nl* nl) { return nl ? nl->j1.get() : nullptr; }
const sg_op* sg_nl_jac_op(const sg_nl* nl) { return nl ? nl->jac.get() : nullptr; }

size_t newton_workspace_bytes(const sg_nl* nl, int n_sub, sg_coarse_kind coarse, int restart) {
    if (!nl || restart < 1) return 0;
    return newton_ws(nl->n, nl->P, n_sub, coarse, restart);
}

int newton_solve(sg_nl* nl, const int32_t* owner, int n_sub, int overlap, sg_prec prec,
                 sg_coarse_kind coarse, double* U, const sg_newton_opts* opts,
                 sg_newton_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nl && owner && U && opts, "null argument");
        check_device(nl->device);
        SG_REQUIRE(opts->max_steps >= 0, "max_steps must be >= 0");
        SG_REQUIRE(opts->tol > 0.0, "tol must be > 0");
        SG_REQUIRE(opts->restart >= 1 && opts->restart <= 64, "restart outside [1,64]");
        SG_REQUIRE(opts->max_it >= 1, "max_it must be >= 1");
        SG_REQUIRE(opts->eta_max > 0.0 && opts->eta_max < 1.0, "eta_max outside (0,1)");
        SG_REQUIRE(opts->amg_rebuild >= 0, "amg_rebuild must be >= 0");
        SG_REQUIRE(opts->method == SG_NEWTON || opts->method == SG_PICARD,
                   "method must be SG_NEWTON or SG_PICARD");
        SG_REQUIRE(opts->du_tol >= 0.0, "du_tol must be >= 0");
        SG_REQUIRE(opts->ras_path >= -1 && opts->ras_path <= 3, "ras_path outside [-1,3]");
        const bool picard = opts->method == SG_PICARD;
        const size_t need = newton_ws(nl->n, nl->P, n_sub, coarse, opts->restart);
        if (!ws || ws_bytes < need)
            SG_THROW(SG_ERR_WORKSPACE, "newton workspace too small (%zu < %zu)", ws_bytes, need);
        hipStream_t s = as_stream(stream);
        const int64_t N = (int64_t)nl->n * nl->P;
        const size_t vb = align_up((size_t)N * 8);
        char* p = reinterpret_cast<char*>(ws);
        double* R = reinterpret_cast<double*>(p);
        double* D = reinterpret_cast<double*>(p + vb);
        double* Ut = reinterpret_cast<double*>(p + 2 * vb);
        double* Rt = reinterpret_cast<double*>(p + 3 * vb);
        double* part = reinterpret_cast<double*>(p + 4 * vb);
        double* scal = reinterpret_cast<double*>(p + 4 * vb + align_up(kMaxRedBlocks * 8));
        char* kws = p + 4 * vb + align_up(kMaxRedBlocks * 8) + 256;
        const size_t kws_bytes = ws_bytes - (size_t)(kws - p);

        using clock = std::chrono::steady_clock;
        auto ms_since = [](clock::time_point a) {
            return std::chrono::duration<double, std::milli>(clock::now() - a).count();
        };
        const auto t_all = clock::now();
        double ms_eval = 0.0, ms_setup = 0.0, ms_krylov = 0.0;
        int hist = 0, kits = 0, steps = 0;
        auto push = [&](double rel, int its) {
            if (stats && stats->history && hist < stats->history_cap) stats->history[hist] = rel;
            if (stats && stats->krylov_its_per_step && hist > 0 && hist - 1 < stats->history_cap)
                stats->krylov_its_per_step[hist - 1] = its;
            ++hist;
        };

        auto t0 = clock::now();
        nl_eval(nl, U, R, s);
        double rn = std::sqrt(host_dot(N, R, R, part, scal, s));
        ms_eval += ms_since(t0);
        const double fn0 = std::sqrt(host_dot(N, nl->B.p, nl->B.p, part, scal, s));
        const double Fn = fn0 > 0.0 ? fn0 : rn;
        if (!std::isfinite(rn)) SG_THROW(SG_ERR_NUMERIC, "initial residual is not finite");
        bool converged = (Fn == 0.0) || rn / Fn <= opts->tol;
        push(Fn > 0.0 ? rn / Fn : 0.0, 0);
        std::unique_ptr<sg_ras, RasDel> ras;
        std::unique_ptr<sg_amg, AmgDel> amg;
        // the linear operator of a step: the Jacobian (Newton) or the secant
        // operator K1(U) with A(U) = K1(U) U (Picard)
        sg_op* Jop = picard ? nl->j1.get() : nl->jac.get();
        LinOp J;
        J.kron = Jop;
        J.n = nl->n;
        J.P = nl->P;
        double last_lambda = 0.0, last_du = 0.0;
        while (!converged && steps < opts->max_steps) {
            // forcing term, safeguarded against solving the correction more
            // accurately than the final tolerance needs
            double eta = std::max(1e-12, std::min(opts->eta_max, rn / Fn));
            eta = std::min(opts->eta_max, std::max(eta, 0.5 * opts->tol * Fn / rn));
            // preconditioner of the current Jacobian
            t0 = clock::now();
            if (!ras) {
                sg_ras* r = nullptr;
                check_status(ras_setup(nl->j1.get(), owner, n_sub, overlap, prec, &r, stream),
                             "ras_setup");
                ras.reset(r);
                // the apply path chosen once; a refactorisation keeps it (and
                // rebuilds the dense rows of a dense path)
                if (opts->ras_path < 0)
                    check_status(ras_autotune(ras.get(), 3, nullptr, stream), "ras_autotune");
                else if (opts->ras_path > 0)
                    check_status(ras_select(ras.get(), opts->ras_path, stream), "ras_select");
            } else {
                check_status(ras_refactor(ras.get(), nl->j1.get(), stream), "ras_refactor");
            }
            const bool rebuild = !amg || (opts->amg_rebuild > 0 && steps % opts->amg_rebuild == 0);
            if (coarse != SG_COARSE_NONE && rebuild) {
                amg.reset();
                sg_amg* a = nullptr;
                check_status(amg_setup(Jop, ras.get(), coarse, prec, &a, stream), "amg_setup");
                amg.reset(a);
            }
            ms_setup += ms_since(t0);
            // correction: J D = R to relative tolerance eta
            t0 = clock::now();
            nl_fill_kernel<<<grid1d(N), 256, 0, s>>>(N, 0.0, D);
            HIP_LAUNCH_OK();
            sg_krylov_opts ko{};
            ko.restart = opts->restart;
            ko.max_it = opts->max_it;
            ko.rtol = eta;
            ko.omega = opts->omega;
            ko.use_graph = opts->use_graph;
            ko.ortho = opts->ortho;
            sg_krylov_stats ks{};
            const int kst = fgmres_core(J, Jop, nl->device, ras.get(), amg.get(), R, D, &ko, &ks,
                                        kws, kws_bytes, s);
            if (kst < 0) return kst;
            kits += ks.iterations;
            ms_krylov += ms_since(t0);
            // backtracking on ||R|| (Newton); the full step (Picard)
            t0 = clock::now();
            double lam = 1.0, rt = 0.0;
            for (int ls = 0; ls < (picard ? 1 : 10); ++ls) {
                nl_axpy_kernel<<<grid1d(N), 256, 0, s>>>(N, lam, U, D, Ut);
                HIP_LAUNCH_OK();
                nl_eval(nl, Ut, Rt, s);
                rt = std::sqrt(host_dot(N, Rt, Rt, part, scal, s));
                if (picard || (std::isfinite(rt) && rt <= (1.0 - 1e-4 * lam) * rn) || ls == 9) break;
                lam *= 0.5;
            }
            if (!std::isfinite(rt)) SG_THROW(SG_ERR_NUMERIC, "residual is not finite");
            HIP_OK(hipMemcpyAsync(U, Ut, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
            std::swap(R, Rt);
            rn = rt;
            ms_eval += ms_since(t0);
            ++steps;
            last_lambda = lam;
            push(rn / Fn, ks.iterations);
            converged = rn / Fn <= opts->tol;
            if (opts->du_tol > 0.0) {
                // relative size of the update, ||lambda D|| / ||U||
                const double dn = lam * std::sqrt(host_dot(N, D, D, part, scal, s));
                const double un = std::sqrt(host_dot(N, U, U, part, scal, s));
                last_du = un > 0.0 ? dn / un : dn;
                converged = converged || last_du <= opts->du_tol;
            }
        }
        HIP_OK(hipStreamSynchronize(s));
        if (stats) {
            stats->steps = steps;
            stats->krylov_its = kits;
            stats->converged = converged ? 1 : 0;
            stats->relres = Fn > 0.0 ? rn / Fn : 0.0;
            stats->last_lambda = last_lambda;
            stats->last_du = last_du;
            stats->ms_total = ms_since(t_all);
            stats->ms_eval = ms_eval;
            stats->ms_setup = ms_setup;
            stats->ms_krylov = ms_krylov;
            stats->history_len = hist < stats->history_cap ? hist : stats->history_cap;
        }
        return converged ? SG_OK : SG_NOT_CONVERGED;
    });
}

void sg_destroy_nl(sg_nl* nl) {
    if (!nl) return;
    graph_cache_purge(nl->jac.get());
    graph_cache_purge(nl->j1.get());
    delete nl;
}

}  // extern "C"
