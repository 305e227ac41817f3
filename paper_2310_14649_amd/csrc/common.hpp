// Internal helpers shared by the sgsolve translation units: error
// propagation across the C ABI, device buffers, and the handle layouts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sgsolve.h"

namespace sg {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const char* msg);

#define SG_THROW(code, ...)                                                  \
    do {                                                                     \
        char _b[512];                                                        \
        std::snprintf(_b, sizeof(_b), __VA_ARGS__);                          \
        throw ::sg::Error((code), _b);                                       \
    } while (0)

#define SG_REQUIRE(cond, ...)                                                \
    do {                                                                     \
        if (!(cond)) SG_THROW(SG_ERR_INVALID_ARG, __VA_ARGS__);              \
    } while (0)

#define HIP_OK(expr)                                                         \
    do {                                                                     \
        hipError_t _e = (expr);                                              \
        if (_e != hipSuccess)                                                \
            SG_THROW(SG_ERR_HIP, "%s failed: %s (%s:%d)", #expr,             \
                     hipGetErrorString(_e), __FILE__, __LINE__);             \
    } while (0)

#define HIP_LAUNCH_OK() HIP_OK(hipGetLastError())

// Run `body` and translate exceptions into status codes at the ABI edge.
template <class F>
int guarded(F&& body) {
    try {
        return body();
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return SG_ERR_INVALID_ARG;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return SG_ERR_INVALID_ARG;
    }
}

// memory.hip: every device buffer of the library (hipMalloc, the caller's
// allocator or the caller's arena; see sg_set_allocator / sg_set_arena)
void* device_alloc(size_t bytes);
void device_free(void* p);

// Owning device allocation.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) p = static_cast<T*>(device_alloc(count * sizeof(T)));
    }
    void release() {
        if (p) device_free(p);
        p = nullptr;
        n = 0;
    }
    void upload(const T* h, size_t count, hipStream_t s) {
        if (count > n) alloc(count);
        if (count) HIP_OK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
    void download(T* h, size_t count, hipStream_t s) const {
        if (count) HIP_OK(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
    size_t bytes() const { return n * sizeof(T); }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int current_device() {
    int d = 0;
    HIP_OK(hipGetDevice(&d));
    return d;
}

inline void check_device(int dev) {
    if (current_device() != dev)
        SG_THROW(SG_ERR_INVALID_ARG, "handle created on device %d used on device %d", dev,
                 current_device());
}

// Triple-product table on the device, sorted by k: for output mode k the
// triples are [kptr[k], kptr[k+1]); tij packs i*P + j; tval = m_ijk.
struct TriplesDev {
    int P = 0, L = 0, T = 0;
    DevBuf<int32_t> kptr, tij;
    DevBuf<double> tval;
    // Schedule of the wide matvec (L > 32 or P > 64): the k-sorted triples cut
    // into 64 equal lane chunks; a lane flushes its running sum into a slot at
    // the end of every run of equal k, and the slots of k are contiguous
    // ([slot_ptr[k], slot_ptr[k+1])), so y_k sums them in a fixed order.
    // sched packs i (16 bits) | j << 16 (7 bits) | slot << 23 (8 bits) | flush << 31.
    int nslot = 0;
    DevBuf<int32_t> lane_ptr, slot_ptr;
    DevBuf<uint32_t> sched;
};

// A "Kronecker-sum" operator Y = sum_i A_i X G_i on a CSR pattern with L
// values per entry (entry-major).  Used for the fine SG operator and for the
// first coarse level.
struct KronCsr {
    int n = 0;
    int64_t nnz = 0;
    int max_row = 0;
    const int32_t* rowptr = nullptr;   // device, n+1 (int32: nnz < 2^31)
    const int32_t* col = nullptr;      // device
    const double* vals = nullptr;      // device, nnz*L
    // optional wave-tiled ELL copy used by the specialised kernels
    int spec = -1;                     // specialisation id, -1 = generic kernel
    int ell_S = 0, ell_RW = 0;         // slots per row, rows per tile
    const int32_t* ecol = nullptr;     // [tiles][S][RW]
    const double* evals = nullptr;     // [tiles][S][L][RW]
    // optional staged copy used by the split kernels (id -1 = none): per
    // block of rows, the runs of neighbour rows staged in LDS, and each
    // entry's column as an index into that staging area
    int split = -1, split_kt = 0;      // split_kt: tiles of 64 rows per work-group
    int group = -1;                    // grouped kernel id (one tile per work-group), -1 = none
    const int32_t* sruns = nullptr;    // [blocks][2*kRuns+1]
    const int16_t* sslot = nullptr;    // [tiles][S][64]
    const double* svals = nullptr;     // [tiles][S][L][64]
    // matrix-free apply of the split kernel (lattice meshes): the K values of
    // a row are formed from the fields of its six elements
    bool mf = false;
    int mf_N = 0;                      // cells per side of the lattice
    const int16_t* sdir = nullptr;     // [tiles][S][64] staging index per stencil direction
    const double* ef = nullptr;        // [n_tri][M+1]: c0, g_1..g_M at the centroid
    const double* ek6 = nullptr;       // [n_tri][6] local stiffness (00,11,22,01,12,02) or null
    double ekL[6] = {}, ekU[6] = {};   // the two element matrices of a uniform lattice
    // row-tiled kernel for wide input bases (one lane per row, tiles of 64
    // rows; staging in sruns / sslot, values in svals): per (chunk of input
    // terms, wave) a list of (i - chunk start) | j << 8 | mode slot << 16
    // with its m_ijk, and the output mode of every (wave, slot) (-1 = none)
    bool rowt = false;
    int rt_nch = 0;
    const int32_t* rt_lptr = nullptr;  // [nch][waves] + 1
    const uint32_t* rt_lij = nullptr;
    const double* rt_lm = nullptr;
    const int32_t* rt_wk = nullptr;    // [waves][slots]
};

}  // namespace sg

struct sg_basis {
    int M = 0, p_in = 0, p = 0, P = 0, L = 0, T = 0;
    std::vector<int32_t> alpha;                 // P*M
    std::vector<int32_t> ti, tj, tk;            // sorted by (k, i, j)
    std::vector<double> tv;
    std::vector<double> afact;                  // <Psi_k^2> = alpha!
};

struct sg_op {
    int device = 0;
    int n = 0, P = 0, L = 0, M = 0;
    int64_t nnz = 0;
    int max_row = 0;
    sg::DevBuf<int32_t> rowptr, col;
    sg::DevBuf<double> vals;         // nnz*L
    sg::DevBuf<double> F;            // n
    sg::DevBuf<double> afact;        // P
    sg::TriplesDev tr;
    int spec = -1, ell_S = 0, ell_RW = 0;
    sg::DevBuf<int32_t> ecol;
    sg::DevBuf<double> evals;
    int split = -1;
    int group = -1;                    // grouped kernel (staging in sruns[0], sslot[0], svals)
    int split_var = 0;                 // selected tile count: 1, 2, 4 tiles for 0, 1, 2
    bool split_fits[3] = {false, false, false};
    sg::DevBuf<int32_t> sruns[3];
    sg::DevBuf<int16_t> sslot[3];
    sg::DevBuf<double> svals;
    // matrix-free apply (sg_matvec_matrix_free), for meshes that are the
    // structured N x N lattice of "/"-cut squares (jittered or not)
    int lattice_N = 0;                 // 0: not a lattice
    // values fixed after construction (sg_assemble, coarse operators); the
    // operators of a nonlinear problem change at every evaluation
    bool fixed_values = false;
    bool mf_on = false, mf_uniform = false;
    bool mf_fits[3] = {false, false, false};
    sg::DevBuf<double> mf_ef, mf_ek6;
    sg::DevBuf<int16_t> mf_sdir[3];
    double mf_ekL[6] = {}, mf_ekU[6] = {};
    // row-tiled kernel (wide input bases): built when the pattern and the
    // basis fit it, used while rt_on; rt_ent maps its value slots to CSR
    // entries, for refreshing svals when the values change
    bool rt_built = false, rt_on = false;
    int rt_nch = 0;
    sg::DevBuf<int32_t> rt_lptr, rt_wk;
    sg::DevBuf<uint32_t> rt_lij;
    sg::DevBuf<double> rt_lm;
    sg::DevBuf<int64_t> rt_ent;
    // host copies used by the setup of the preconditioner
    std::vector<int32_t> h_rowptr, h_col;
    std::vector<int64_t> h_graph_ptr;           // mesh graph (overlap growth)
    std::vector<int32_t> h_graph_col;
    std::vector<double> h_afact;
    sg_basis basis;

    sg::KronCsr csr() const {
        sg::KronCsr k;
        k.n = n; k.nnz = nnz; k.max_row = max_row;
        k.rowptr = rowptr.p; k.col = col.p; k.vals = vals.p;
        k.spec = spec; k.ell_S = ell_S; k.ell_RW = ell_RW; k.ecol = ecol.p; k.evals = evals.p;
        k.split = split; k.split_kt = 1 << split_var; k.group = group;
        k.sruns = sruns[split_var].p; k.sslot = sslot[split_var].p; k.svals = svals.p;
        k.mf = mf_on && split >= 0;
        if (k.mf) {
            k.mf_N = lattice_N; k.sdir = mf_sdir[split_var].p; k.ef = mf_ef.p;
            k.ek6 = mf_uniform ? nullptr : mf_ek6.p;
            for (int q = 0; q < 6; ++q) { k.ekL[q] = mf_ekL[q]; k.ekU[q] = mf_ekU[q]; }
        }
        k.rowt = rt_built && rt_on && split < 0 && group < 0;
        if (k.rowt) {
            k.sruns = sruns[0].p; k.sslot = sslot[0].p; k.svals = svals.p;
            k.rt_nch = rt_nch; k.rt_lptr = rt_lptr.p; k.rt_lij = rt_lij.p; k.rt_lm = rt_lm.p;
            k.rt_wk = rt_wk.p;
        }
        return k;
    }
};

namespace sg {
// matvec.hip: Y = alpha * (sum_i A_i X G_i) + beta * C  (C may equal Y).
void kron_matvec(const KronCsr& A, int L, const TriplesDev& tr, const double* X, double* Y,
                 double alpha, double beta, const double* C, hipStream_t s);
// matvec.hip: pick a specialised kernel for this basis/pattern and build its
// wave-tiled ELL copy of the values (no-op when none applies).
void build_ell(sg_op* op, hipStream_t s);
// matvec.hip: build the row-tiled kernel's staging, lists and value copy
// when the basis is wide (L > 32) and the pattern fits; false otherwise.
bool build_row_tiled(sg_op* op, hipStream_t s);
// matvec.hip: copy op->vals into the row-tiled value layout (after the
// values change; no-op when the kernel is not built).
void refresh_row_tiled(sg_op* op, hipStream_t s);
// triples.hip: upload a basis' triple table.
void upload_triples(const sg_basis& b, TriplesDev& tr, hipStream_t s);
// triples.hip: graded multi-indices of total degree <= p (count in `count`).
void enumerate(int M, int p, std::vector<int32_t>& alpha, int& count);
int binom(int n, int k);
// triples.hip: non-zero <Psi_a Psi_b Psi_c> for a < na, b < nb, c < nc of
// the degree-`deg` basis, sorted by (c, a, b).
struct SparseTriples {
    std::vector<int32_t> a, b, c;
    std::vector<double> v;
};
void sparse_triples(int M, int deg, int na, int nb, int nc, SparseTriples& out);
}  // namespace sg

namespace sg {
// assemble.hip: mesh checks, the P1 pattern with the element contributions
// of every entry (cref = t*9 + la*3 + lb, in a fixed order), the mesh graph,
// per-element geometry and input PCE, and the load vector of f = 1.
struct MeshPattern {
    std::vector<int32_t> rowptr, col, cref;
    std::vector<int64_t> cptr;
    int max_row = 0;
    std::vector<int64_t> graph_ptr;
    std::vector<int32_t> graph_col;
};
void validate_mesh(int n_vert, const double* xy, int n_tri, const int32_t* tri,
                   const int32_t* dof, int n);
// prune: leave out off-diagonal entries whose geometric weight is exactly 0
// in every element sharing the edge.
void mesh_pattern(int n_vert, const double* xy, int n_tri, const int32_t* tri, const int32_t* dof,
                  int n, bool prune, MeshPattern& out);
struct ElementData {
    DevBuf<double> ek;      // [n_tri][3][3] |T| grad phi_a . grad phi_b
    DevBuf<double> ec;      // [n_tri][L] input PCE coefficients at the centroid
    DevBuf<double> earea;   // [n_tri]
    DevBuf<double> ef;      // [n_tri][M+1]: c0 = exp(g0 + |g|^2/2), g_1..g_M
};
// Cells per side N when the mesh is the structured lattice: (N+1)^2
// vertices v(i,j) = j(N+1) + i, element 2(jN + i) = (v(i,j), v(i+1,j),
// v(i+1,j+1)) and 2(jN + i) + 1 = (v(i,j), v(i+1,j+1), v(i,j+1)), unknown
// (j-1)(N-1) + (i-1) at interior vertices; 0 otherwise.
int lattice_cells(int n_vert, int n_tri, const int32_t* tri, const int32_t* dof, int n);
// An SG operator sum_i K_i (x) G_i from a CSR pattern with L values per entry
// (entry-major, host) and its mesh graph (for overlap growth), e.g. a
// Galerkin coarse operator; no load vector.
sg_op* make_csr_op(const sg_basis& b, int n, const std::vector<int32_t>& rowptr,
                   const std::vector<int32_t>& col, const std::vector<double>& vals,
                   const std::vector<int64_t>& graph_ptr, const std::vector<int32_t>& graph_col,
                   hipStream_t s);
void element_data(const sg_basis& b, int n_vert, const double* xy, int n_tri, const int32_t* tri,
                  const double* g0, const double* g, ElementData& out, hipStream_t s);
void load_vector(int n, const int32_t* rowptr, const int32_t* col, const int64_t* cptr,
                 const int32_t* cref, const double* earea, double* F, hipStream_t s);
}  // namespace sg

struct sg_ras;
struct sg_amg;
namespace sg {
// The operator FGMRES and the two-grid cycle apply: the Kronecker-sum SG
// operator of an sg_op (the linear operator, or a Newton Jacobian whose
// input terms are its degree-2p coefficient fields).
struct LinOp {
    const sg_op* kron = nullptr;
    int n = 0, P = 0;
};
// Y = alpha * (A X) + beta * C  (C may equal Y; X must not alias Y)
void linop_apply(const LinOp& A, const double* X, double* Y, double alpha, double beta,
                 const double* C, hipStream_t s);
// ras.hip: Z[owned] = beta * Z[owned] + omega * RAS(R)[owned]
// cadd, cown (fused path only, beta = 1): also add cadd[cown[a]] to row a
void ras_apply_ex(const sg_ras* r, const double* R, double* Z, double omega, double beta,
                  hipStream_t s, const double* cadd = nullptr, const int32_t* cown = nullptr);
bool ras_can_add_coarse(const sg_ras* r);
const std::vector<int32_t>& ras_owner(const sg_ras* r);
int ras_nsub(const sg_ras* r);
int ras_device(const sg_ras* r);
int ras_n(const sg_ras* r);
// coarse.hip
void coarse_restrict(const sg_amg* a, const double* R, double* rc, hipStream_t s);
void coarse_prolong_add(const sg_amg* a, const double* ec, double* Y, hipStream_t s);
void coarse_solve(const sg_amg* a, const double* b, double* x, hipStream_t s);
// T -= (A Z) e_c for the operator the coarse space was built from, where the
// product touches only the rows next to a subdomain interface or the
// boundary; false (nothing done) when `op` is not that operator.
bool coarse_residual_update(const sg_amg* a, const sg_op* op, const double* ec, double* T,
                            hipStream_t s);
// the coarse space holds A Z for `op` (coarse_residual_update applies)
bool coarse_has_az(const sg_amg* a, const sg_op* op);
// the subdomain of every fine node for a Nicolaides space (device), else NULL
const int32_t* coarse_owner_dev(const sg_amg* a);
// true when the coarse solve is an inner Krylov iteration (host-synchronous,
// so the Arnoldi step that contains it is not captured into a graph)
bool inner_active(const sg_amg* a);
int amg_nsub(const sg_amg* a);
bool amg_is_geometric(const sg_amg* a);
int amg_fine_n(const sg_amg* a);
// krylov.hip: drop cached Arnoldi-step graphs that reference a handle
void graph_cache_purge(const void* handle);
int amg_device(const sg_amg* a);
// krylov.hip
constexpr int kMaxRedBlocks = 1024;
inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }
// synchronous dot product; part: kMaxRedBlocks doubles, scal: 1 double
double host_dot(int64_t N, const double* x, const double* y, double* part, double* scal,
                hipStream_t s);
// workspace of fgmres_core with ns coarse subdomains (ns < 0: no coarse solve)
size_t fgmres_ws_ns(int n, int P, int ns, int restart);
size_t fgmres_ws_np(int n, int P, const sg_amg* amg, int restart);
double smoother_damping_core(const LinOp& A, const sg_ras* ras, int its, char* ws, size_t ws_bytes,
                             hipStream_t s, double* rho_out);
// key_op identifies the operator in the graph cache
int fgmres_core(const LinOp& A, const void* key_op, int device, const sg_ras* ras,
                const sg_amg* amg, const double* b, double* x, const sg_krylov_opts* opts,
                sg_krylov_stats* stats, void* ws, size_t ws_bytes, hipStream_t s);
}  // namespace sg
