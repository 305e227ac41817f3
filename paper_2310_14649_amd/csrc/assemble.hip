// Assembly of the SG operator (Eq. Galerkin_L_exp): one P1 stiffness matrix
// per input PCE term on a shared CSR pattern, with the log-normal input PCE
// (Eq. inputlogn) evaluated at element centroids on the device.
//
// Host work is integer/combinatorial: the CSR pattern, the list of element
// contributions of every entry (so the device sums them in a fixed order,
// without atomics), and the mesh graph used later to grow subdomain
// overlaps.  An off-diagonal entry is left out of the pattern when its
// geometric weight |T| grad phi_a . grad phi_b is exactly zero in every
// element sharing the edge (a right angle opposite the edge, as on the
// hypotenuses of a structured "/" mesh): its value would be 0 for every
// coefficient field.
#include "common.hpp"

#include <algorithm>
#include <numeric>

namespace sg {
namespace {

constexpr int kMaxL = 64;

// Per element: area, local stiffness |T| grad phi_a . grad phi_b (3x3), and
// the input PCE coefficients c_i = c0 prod_m g_m^alpha_m / alpha_m!,
// c0 = exp(g0 + 1/2 sum_m g_m^2).
__global__ void element_kernel(int n_tri, int M, int L, const double* __restrict__ xy,
                               const int32_t* __restrict__ tri, const double* __restrict__ g0,
                               const double* __restrict__ g, const int32_t* __restrict__ alpha,
                               double* __restrict__ ek, double* __restrict__ ec,
                               double* __restrict__ earea, double* __restrict__ ef,
                               int* __restrict__ bad) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
    double x[3] = {xy[2 * v0], xy[2 * v1], xy[2 * v2]};
    double y[3] = {xy[2 * v0 + 1], xy[2 * v1 + 1], xy[2 * v2 + 1]};
    double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    if (!(det > 0.0)) {
        atomicOr(bad, 1);
        det = 1.0;
    }
    double area = 0.5 * det;
    double gx[3], gy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        gx[k] = (y[k1] - y[k2]) / det;
        gy[k] = (x[k2] - x[k1]) / det;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) ek[9 * (int64_t)t + 3 * a + b] = area * (gx[a] * gx[b] + gy[a] * gy[b]);
    earea[t] = area;

    double gm[8];
    double s2 = 0.0;
    for (int m = 0; m < M; ++m) {
        gm[m] = g[(int64_t)m * n_tri + t];
        s2 += gm[m] * gm[m];
    }
    double c0 = exp(g0[t] + 0.5 * s2);
    ef[(int64_t)t * (M + 1)] = c0;
    for (int m = 0; m < M; ++m) ef[(int64_t)t * (M + 1) + 1 + m] = gm[m];
    for (int i = 0; i < L; ++i) {
        double term = c0;
        for (int m = 0; m < M; ++m) {
            int am = alpha[i * M + m];
            for (int e = 1; e <= am; ++e) term *= gm[m] / (double)e;
        }
        ec[(int64_t)t * L + i] = term;
    }
}

// One thread per (entry, input term): fixed-order sum of element contributions.
__global__ void entry_kernel(int64_t nnz, int L, const int64_t* __restrict__ cptr,
                             const int32_t* __restrict__ cref, const double* __restrict__ ek,
                             const double* __restrict__ ec, double* __restrict__ vals) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nnz * L) return;
    int64_t e = idx / L;
    int i = (int)(idx - e * L);
    double acc = 0.0;
    for (int64_t c = cptr[e]; c < cptr[e + 1]; ++c) {
        int32_t r = cref[c];
        int32_t t = r / 9, pr = r - 9 * (r / 9);
        acc += ec[(int64_t)t * L + i] * ek[9 * (int64_t)t + pr];
    }
    vals[idx] = acc;
}

// F[a] = sum over elements at a of |T|/3: the diagonal entry's contribution
// list is exactly the list of elements touching a.
__global__ void load_kernel(int n, const int32_t* __restrict__ rowptr,
                            const int32_t* __restrict__ col, const int64_t* __restrict__ cptr,
                            const int32_t* __restrict__ cref, const double* __restrict__ earea,
                            double* __restrict__ F) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double acc = 0.0;
    for (int e = rowptr[a]; e < rowptr[a + 1]; ++e) {
        if (col[e] != a) continue;
        for (int64_t c = cptr[e]; c < cptr[e + 1]; ++c) acc += earea[cref[c] / 9] / 3.0;
    }
    F[a] = acc;
}

__global__ void rhs_kernel(int n, int P, const double* __restrict__ F, double* __restrict__ B) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * P) return;
    int64_t a = idx / P;
    int k = (int)(idx - a * P);
    B[idx] = (k == 0) ? F[a] : 0.0;
}

}  // namespace
}  // namespace sg

namespace sg {

void validate_mesh(int n_vert, const double* xy, int n_tri, const int32_t* tri,
                   const int32_t* dof, int n) {
    SG_REQUIRE(xy && tri && dof, "null mesh argument");
    SG_REQUIRE(n_vert > 0 && n_tri > 0 && n > 0, "empty mesh");
    for (int v = 0; v < n_vert; ++v)
        SG_REQUIRE(dof[v] >= -1 && dof[v] < n, "dof[%d]=%d outside [-1,%d)", v, dof[v], n);
    std::vector<char> seen(n, 0);
    for (int v = 0; v < n_vert; ++v)
        if (dof[v] >= 0) {
            SG_REQUIRE(!seen[dof[v]], "dof %d used twice", dof[v]);
            seen[dof[v]] = 1;
        }
    for (int a = 0; a < n; ++a) SG_REQUIRE(seen[a], "unknown %d has no vertex", a);
    for (int64_t t = 0; t < (int64_t)n_tri * 3; ++t)
        SG_REQUIRE(tri[t] >= 0 && tri[t] < n_vert, "tri entry %lld out of range", (long long)t);
}

void mesh_pattern(int n_vert, const double* xy, int n_tri, const int32_t* tri, const int32_t* dof,
                  int n, bool prune, MeshPattern& out) {
    (void)n_vert;
    struct Contrib { int64_t key; int32_t ref; bool keep; };
    std::vector<Contrib> cs;
    cs.reserve((size_t)n_tri * 9);
    std::vector<int64_t> gkeys;
    gkeys.reserve((size_t)n_tri * 6);
    for (int t = 0; t < n_tri; ++t) {
        int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int la = 0; la < 3; ++la) {
            int da = dof[v[la]];
            if (da < 0) continue;
            for (int lb = 0; lb < 3; ++lb) {
                int db = dof[v[lb]];
                if (db < 0) continue;
                bool keep = true;
                if (la != lb) {
                    if (prune) {
                        int lc = 3 - la - lb;
                        double ax = xy[2 * v[la]] - xy[2 * v[lc]], ay = xy[2 * v[la] + 1] - xy[2 * v[lc] + 1];
                        double bx = xy[2 * v[lb]] - xy[2 * v[lc]], by = xy[2 * v[lb] + 1] - xy[2 * v[lc] + 1];
                        keep = (ax * bx + ay * by) != 0.0;
                    }
                    gkeys.push_back((int64_t)da * n + db);
                }
                cs.push_back({(int64_t)da * n + db, t * 9 + la * 3 + lb, keep});
            }
        }
    }
    std::stable_sort(cs.begin(), cs.end(),
                     [](const Contrib& x, const Contrib& y) { return x.key < y.key; });
    out.rowptr.assign(n + 1, 0);
    out.col.clear();
    out.cptr.assign(1, 0);
    out.cref.clear();
    out.max_row = 0;
    size_t i0 = 0;
    while (i0 < cs.size()) {
        size_t i1 = i0;
        bool keep = false;
        while (i1 < cs.size() && cs[i1].key == cs[i0].key) keep |= cs[i1++].keep;
        int r = (int)(cs[i0].key / n), c = (int)(cs[i0].key % n);
        if (keep || r == c) {
            out.col.push_back(c);
            out.rowptr[r + 1]++;
            for (size_t q = i0; q < i1; ++q) out.cref.push_back(cs[q].ref);
            out.cptr.push_back((int64_t)out.cref.size());
        }
        i0 = i1;
    }
    for (int a = 0; a < n; ++a) {
        out.max_row = std::max(out.max_row, out.rowptr[a + 1]);
        out.rowptr[a + 1] += out.rowptr[a];
    }
    SG_REQUIRE((int64_t)out.col.size() < (int64_t)INT32_MAX, "too many non-zeros");
    // mesh graph (all triangle edges between unknowns, pruned or not)
    std::sort(gkeys.begin(), gkeys.end());
    gkeys.erase(std::unique(gkeys.begin(), gkeys.end()), gkeys.end());
    out.graph_ptr.assign(n + 1, 0);
    out.graph_col.resize(gkeys.size());
    for (size_t q = 0; q < gkeys.size(); ++q) {
        out.graph_ptr[gkeys[q] / n + 1]++;
        out.graph_col[q] = (int32_t)(gkeys[q] % n);
    }
    for (int a = 0; a < n; ++a) out.graph_ptr[a + 1] += out.graph_ptr[a];
}

void element_data(const sg_basis& b, int n_vert, const double* xy, int n_tri, const int32_t* tri,
                  const double* g0, const double* g, ElementData& out, hipStream_t s) {
    SG_REQUIRE(b.L <= kMaxL, "L_in=%d exceeds %d", b.L, kMaxL);
    SG_REQUIRE(g0 != nullptr, "g0 is NULL");
    SG_REQUIRE(b.M == 0 || g != nullptr, "g is NULL with M > 0");
    DevBuf<double> d_xy, d_g0, d_g;
    DevBuf<int32_t> d_tri, d_alpha;
    DevBuf<int> d_bad(1);
    out.ek.alloc((size_t)n_tri * 9);
    out.ec.alloc((size_t)n_tri * b.L);
    out.earea.alloc(n_tri);
    out.ef.alloc((size_t)n_tri * (b.M + 1));
    d_xy.upload(xy, (size_t)n_vert * 2, s);
    d_tri.upload(tri, (size_t)n_tri * 3, s);
    d_g0.upload(g0, n_tri, s);
    if (b.M > 0) d_g.upload(g, (size_t)b.M * n_tri, s);
    std::vector<int32_t> alpha_in(b.alpha.begin(), b.alpha.begin() + (size_t)b.L * b.M);
    if (b.M > 0) d_alpha.upload(alpha_in, s);
    HIP_OK(hipMemsetAsync(d_bad.p, 0, sizeof(int), s));
    element_kernel<<<(n_tri + 255) / 256, 256, 0, s>>>(n_tri, b.M, b.L, d_xy.p, d_tri.p, d_g0.p,
                                                        d_g.p, d_alpha.p, out.ek.p, out.ec.p,
                                                        out.earea.p, out.ef.p, d_bad.p);
    HIP_LAUNCH_OK();
    int bad = 0;
    d_bad.download(&bad, 1, s);
    HIP_OK(hipStreamSynchronize(s));
    SG_REQUIRE(!bad, "degenerate or clockwise triangle");
}

int lattice_cells(int n_vert, int n_tri, const int32_t* tri, const int32_t* dof, int n) {
    int N = 0;
    while ((int64_t)(N + 2) * (N + 2) <= n_vert) ++N;
    if ((int64_t)(N + 1) * (N + 1) != n_vert || N < 2) return 0;
    if ((int64_t)n_tri != 2LL * N * N || (int64_t)n != (int64_t)(N - 1) * (N - 1)) return 0;
    auto v = [N](int i, int j) { return j * (N + 1) + i; };
    for (int cj = 0; cj < N; ++cj)
        for (int ci = 0; ci < N; ++ci) {
            const int32_t* a = tri + 6 * ((int64_t)cj * N + ci);
            if (a[0] != v(ci, cj) || a[1] != v(ci + 1, cj) || a[2] != v(ci + 1, cj + 1) ||
                a[3] != v(ci, cj) || a[4] != v(ci + 1, cj + 1) || a[5] != v(ci, cj + 1))
                return 0;
        }
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            const bool in = i > 0 && i < N && j > 0 && j < N;
            if (dof[v(i, j)] != (in ? (j - 1) * (N - 1) + (i - 1) : -1)) return 0;
        }
    return N;
}

sg_op* make_csr_op(const sg_basis& b, int n, const std::vector<int32_t>& rowptr,
                   const std::vector<int32_t>& col, const std::vector<double>& vals,
                   const std::vector<int64_t>& graph_ptr, const std::vector<int32_t>& graph_col,
                   hipStream_t s) {
    SG_REQUIRE((int)rowptr.size() == n + 1 && (size_t)rowptr[n] == col.size() &&
                   vals.size() == col.size() * (size_t)b.L, "inconsistent CSR operator");
    auto op = std::make_unique<sg_op>();
    op->device = current_device();
    op->n = n; op->P = b.P; op->L = b.L; op->M = b.M;
    op->nnz = (int64_t)col.size();
    op->max_row = 0;
    for (int a = 0; a < n; ++a) op->max_row = std::max(op->max_row, rowptr[a + 1] - rowptr[a]);
    op->basis = b;
    op->h_afact = b.afact;
    op->h_rowptr = rowptr;
    op->h_col = col;
    op->h_graph_ptr = graph_ptr;
    op->h_graph_col = graph_col;
    op->fixed_values = true;
    op->rowptr.upload(rowptr, s);
    op->col.upload(col, s);
    op->vals.upload(vals, s);
    op->F.alloc(n);
    HIP_OK(hipMemsetAsync(op->F.p, 0, (size_t)n * 8, s));
    op->afact.upload(b.afact, s);
    upload_triples(b, op->tr, s);
    build_ell(op.get(), s);
    HIP_OK(hipStreamSynchronize(s));
    return op.release();
}

void load_vector(int n, const int32_t* rowptr, const int32_t* col, const int64_t* cptr,
                 const int32_t* cref, const double* earea, double* F, hipStream_t s) {
    load_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, rowptr, col, cptr, cref, earea, F);
    HIP_LAUNCH_OK();
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_assemble(const sg_basis* b, int n_vert, const double* xy, int n_tri, const int32_t* tri,
                const int32_t* dof, int n, const double* g0, const double* g, sg_op** out,
                void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(b && xy && tri && dof && g0 && out, "null argument");
        SG_REQUIRE(b->M == 0 || g != nullptr, "g is NULL with M > 0");
        SG_REQUIRE(b->L <= kMaxL, "L_in=%d exceeds %d", b->L, kMaxL);
        hipStream_t s = as_stream(stream);
        validate_mesh(n_vert, xy, n_tri, tri, dof, n);
        MeshPattern mp;
        mesh_pattern(n_vert, xy, n_tri, tri, dof, n, true, mp);
        const int64_t nnz = (int64_t)mp.col.size();

        auto op = std::make_unique<sg_op>();
        op->device = current_device();
        op->h_graph_ptr = std::move(mp.graph_ptr);
        op->h_graph_col = std::move(mp.graph_col);
        op->n = n; op->P = b->P; op->L = b->L; op->M = b->M;
        op->nnz = nnz; op->max_row = mp.max_row;
        op->basis = *b;
        op->h_afact = b->afact;
        op->h_rowptr = mp.rowptr;
        op->h_col = mp.col;
        op->fixed_values = true;

        // ---- device evaluation ----
        ElementData ed;
        element_data(*b, n_vert, xy, n_tri, tri, g0, g, ed, s);
        DevBuf<int32_t> d_cref;
        DevBuf<int64_t> d_cptr;
        d_cptr.upload(mp.cptr, s);
        d_cref.upload(mp.cref, s);
        op->rowptr.upload(mp.rowptr, s);
        op->col.upload(mp.col, s);
        op->vals.alloc((size_t)nnz * b->L);
        op->F.alloc(n);
        op->afact.upload(b->afact, s);
        int64_t work = nnz * b->L;
        entry_kernel<<<(unsigned)((work + 255) / 256), 256, 0, s>>>(nnz, b->L, d_cptr.p, d_cref.p,
                                                                   ed.ek.p, ed.ec.p, op->vals.p);
        HIP_LAUNCH_OK();
        load_vector(n, op->rowptr.p, op->col.p, d_cptr.p, d_cref.p, ed.earea.p, op->F.p, s);
        upload_triples(*b, op->tr, s);
        build_ell(op.get(), s);
        // lattice meshes keep the element fields and local matrices for the
        // matrix-free apply (sg_matvec_matrix_free)
        op->lattice_N = lattice_cells(n_vert, n_tri, tri, dof, n);
        if (op->lattice_N > 0) {
            std::vector<double> ek((size_t)n_tri * 9);
            ed.ek.download(ek.data(), ek.size(), s);
            HIP_OK(hipStreamSynchronize(s));
            static const int kPair[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {0, 2}};
            std::vector<double> ek6((size_t)n_tri * 6);
            for (int t = 0; t < n_tri; ++t)
                for (int q = 0; q < 6; ++q)
                    ek6[(size_t)t * 6 + q] = ek[(size_t)t * 9 + 3 * kPair[q][0] + kPair[q][1]];
            bool uniform = true;
            for (int t = 2; t < n_tri && uniform; ++t)
                for (int q = 0; q < 6; ++q)
                    if (ek6[(size_t)t * 6 + q] != ek6[(size_t)(t & 1) * 6 + q]) {
                        uniform = false;
                        break;
                    }
            op->mf_uniform = uniform;
            for (int q = 0; q < 6; ++q) {
                op->mf_ekL[q] = ek6[q];
                op->mf_ekU[q] = ek6[6 + q];
            }
            if (!uniform) op->mf_ek6.upload(ek6, s);
            op->mf_ef = std::move(ed.ef);
        }
        HIP_OK(hipStreamSynchronize(s));
        *out = op.release();
        return SG_OK;
    });
}

int sg_op_info(const sg_op* op, int* n, int* P, int* L_in, int64_t* nnz) {
    return guarded([&]() -> int {
        SG_REQUIRE(op != nullptr, "op is NULL");
        if (n) *n = op->n;
        if (P) *P = op->P;
        if (L_in) *L_in = op->L;
        if (nnz) *nnz = op->nnz;
        return SG_OK;
    });
}

int sg_op_rhs(const sg_op* op, double* B, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(op && B, "null argument");
        check_device(op->device);
        int64_t tot = (int64_t)op->n * op->P;
        rhs_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, as_stream(stream)>>>(op->n, op->P,
                                                                                 op->F.p, B);
        HIP_LAUNCH_OK();
        return SG_OK;
    });
}

int sg_op_export(const sg_op* op, int64_t* rowptr, int32_t* col, double* vals) {
    return guarded([&]() -> int {
        SG_REQUIRE(op != nullptr, "op is NULL");
        check_device(op->device);
        if (rowptr)
            for (int a = 0; a <= op->n; ++a) rowptr[a] = op->h_rowptr[a];
        if (col) std::memcpy(col, op->h_col.data(), op->nnz * sizeof(int32_t));
        if (vals) {
            op->vals.download(vals, (size_t)op->nnz * op->L, nullptr);
            HIP_OK(hipDeviceSynchronize());
        }
        return SG_OK;
    });
}

void sg_destroy_op(sg_op* op) {
    sg::graph_cache_purge(op);
    delete op;
}

}  // extern "C"
