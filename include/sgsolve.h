/*
 * sgsolve -- intrusive stochastic Galerkin (SG) solver for the log-normal
 * Poisson problem on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of arXiv 2310.14649, "Multilevel Scalable Solvers for
 * Stochastic Linear and Nonlinear Problems": the Galerkin projection of
 * -div(c(x,xi) grad u) = f onto a Hermite chaos (Sec. 2.1), solved by
 * flexible GMRES preconditioned with a two-grid restricted additive Schwarz
 * cycle whose coarse problem is handled by algebraic multigrid (Sec. 3).
 *
 * Conventions common to every call
 * --------------------------------
 * - All entry points are C functions returning an int status: SG_OK (0),
 *   SG_NOT_CONVERGED (1, outputs and statistics still valid) or a negative
 *   error code.  sg_last_error() returns a thread-local message for the last
 *   failing call of the calling thread.  No C++ exception crosses the ABI.
 * - "device" pointers are HIP device allocations of the current device
 *   (e.g. torch tensors' data_ptr()); "host" pointers are ordinary memory.
 *   The library never frees caller memory.
 * - SG fields are row-major [n x P] FP64 arrays: X[a*P + k] is the k-th PCE
 *   coefficient at unknown a (the vector-PDE layout of Sec. 2.1).
 * - Handles (sg_basis, sg_op, sg_ras, sg_amg) are opaque and own their
 *   device memory (allocated in the *_setup / build / assemble call, freed by
 *   the matching sg_destroy_*).  They must be used on the device that was
 *   current when they were created.
 * - stream is a hipStream_t passed as void* (NULL = default stream).  Calls
 *   that only launch kernels are asynchronous on that stream; setup calls and
 *   solve calls synchronise the stream before returning.
 * - Calls sharing a handle must not run concurrently on different streams.
 */
#ifndef SGSOLVE_H
#define SGSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SG_OK = 0,
    SG_NOT_CONVERGED = 1,
    SG_ERR_INVALID_ARG = -1,   /* bad size, null pointer, inconsistent handles */
    SG_ERR_HIP = -2,           /* a HIP runtime call failed                     */
    SG_ERR_NUMERIC = -3,       /* non-SPD local block, NaN/Inf in a reduction   */
    SG_ERR_UNSUPPORTED = -4,   /* a size beyond a compiled limit                */
    SG_ERR_WORKSPACE = -5      /* workspace too small                           */
};

typedef enum { SG_FP64 = 0, SG_FP32 = 1, SG_BF16 = 2 } sg_prec;

typedef enum {
    SG_COARSE_NONE = 0,        /* one-level RAS only                             */
    SG_COARSE_MEAN_EXACT = 1,  /* (C_0 (x) G_0)^{-1}: exact mean-based coarse     */
    SG_COARSE_AMG = 2,         /* one smoothed-aggregation V(1,1) cycle on A_c    */
    SG_COARSE_GEOMETRIC = 3    /* coarser lattice, A_c = P_0^T A P_0, inner FGMRES */
                               /* (amg_setup_geometric only)                     */
} sg_coarse_kind;

/* Local solves of the RAS subdomains (ras_set_local). */
typedef enum {
    SG_LOCAL_MEAN = 0,   /* mean-based: (R_s A_0 R_s^T)^{-1} (x) G_0^{-1}                  */
    SG_LOCAL_KRON = 1    /* Kronecker (Ullmann): (R_s K_0 R_s^T)^{-1} (x) Gt^{-1}           */
} sg_local_kind;

/* The coarse problem of the two-grid cycle solved by an inner Krylov method
 * (Sec. 3: the variants that solve the coarse problem inexactly by GMRES). */
typedef enum {
    SG_INNER_NONE = 0,       /* the coarse kind's own solve (one V-cycle)           */
    SG_INNER_GMRES_AMG = 1,  /* 2GV3: GMRES on A_c preconditioned by one V-cycle    */
    SG_INNER_GMRES_BJ = 2    /* 2GV2: GMRES on A_c preconditioned by block Jacobi   */
} sg_inner_kind;

typedef struct sg_basis sg_basis;
typedef struct sg_op sg_op;
typedef struct sg_ras sg_ras;
typedef struct sg_amg sg_amg;

const char* sg_last_error(void);
int sg_version(void);

/* ------------------------------------------------------------------------
 * Device memory.  Every device buffer a handle holds (operators, factors,
 * hierarchies, internal workspaces of setup, networks), and every temporary
 * buffer of a setup call, is taken from one source, chosen process-wide:
 *   - hipMalloc / hipFree (the default);
 *   - the caller's functions (sg_set_allocator): alloc(bytes, device, ctx)
 *     returns a 256-byte aligned device pointer on `device` or NULL (the
 *     call then fails with SG_ERR_WORKSPACE); release(ptr, bytes, device,
 *     ctx) takes it back when the handle is destroyed or the temporary
 *     dropped.  A stream-ordered allocator (e.g. a framework's caching
 *     allocator) must order the release after the library's work: destroy
 *     handles only after their work has finished;
 *   - a caller-owned arena (sg_set_arena): base (256-byte aligned device
 *     memory of the current device) and bytes; buffers are cut from it in
 *     order and never reused until sg_arena_reset (which needs every buffer
 *     cut from it released, i.e. the handles destroyed).  An allocation
 *     beyond the arena fails with SG_ERR_WORKSPACE and the setup call
 *     releases what it had taken.
 * The bytes a sequence of setup calls needs are found by running it once
 * and reading the peak (sg_memory_stats: live bytes held by the library,
 * their peak since sg_memory_reset_peak, and the bytes cut from the arena).
 * A buffer goes back to the source it came from even if the source changed
 * meanwhile.  sg_set_allocator(NULL, NULL, NULL) restores hipMalloc and
 * sg_set_arena(NULL, 0) leaves arena mode.  Not to be called while another
 * thread is inside the library.  Pinned host memory (a few residual
 * estimates) still comes from hipHostMalloc.
 * ---------------------------------------------------------------------- */
typedef void* (*sg_device_alloc_fn)(size_t bytes, int device, void* ctx);
typedef void (*sg_device_free_fn)(void* ptr, size_t bytes, int device, void* ctx);
int sg_set_allocator(sg_device_alloc_fn alloc, sg_device_free_fn release, void* ctx);
int sg_set_arena(void* base, size_t bytes);
int sg_arena_reset(void);
int sg_memory_stats(int64_t* live_bytes, int64_t* peak_bytes, int64_t* arena_used);
int sg_memory_reset_peak(void);

/* ------------------------------------------------------------------------
 * sg_build_triples -- Hermite chaos basis and the triple-product tensor
 * m_ijk = <Psi_i Psi_j Psi_k> of Eq. Galerkin_L_exp, keeping only non-zero
 * entries (Sec. 2.1: only the non-zero multiplication-tensor entries are
 * stored).  Psi_alpha = prod_m He_{alpha_m}(xi_m), probabilists' Hermite,
 * un-normalised (<Psi_alpha^2> = alpha!).  Multi-indices with |alpha| <= p
 * are ordered by total degree, then descending lexicographically; the input
 * basis (|alpha| <= p_in, L_in = (M+p_in)!/(M! p_in!) terms, the count
 * under Eq. inputpc) is the prefix of the output basis (P terms).
 * i runs over the input basis, j and k over the output basis.
 * The values are integers (exact in FP64), computed on the device.
 * Limits: 0 <= M <= 8, 0 <= p_in <= p_out <= 4, P <= 128.
 * Errors: SG_ERR_INVALID_ARG for out-of-range arguments.
 * ---------------------------------------------------------------------- */
int sg_build_triples(int M, int p_in, int p_out, sg_basis** out);
int sg_basis_info(const sg_basis* b, int* P, int* L_in, int* n_triples);
/* host outputs: alpha [P*M] int32, ijk [T*3] int32 (i,j,k), val [T] FP64.
 * Triples are sorted by k, then i, then j.  Any pointer may be NULL. */
int sg_basis_export(const sg_basis* b, int32_t* alpha, int32_t* ijk, double* val);
void sg_destroy_basis(sg_basis* b);

/* ------------------------------------------------------------------------
 * sg_assemble -- the SG operator of Eq. Galerkin_L_exp on a P1 mesh.
 * Inputs (all host, copied):
 *   xy  [n_vert*2]   vertex coordinates
 *   tri [n_tri*3]    counter-clockwise vertex triples
 *   dof [n_vert]     unknown number of each vertex, -1 = Dirichlet (u = 0)
 *   n                number of unknowns (max dof + 1)
 *   g0  [n_tri]      mean of the Gaussian field at element centroids
 *   g   [M*n_tri]    KL modes g_m at element centroids (row m contiguous)
 * The device evaluates the log-normal input PCE (Eq. inputlogn, with the
 * mean exp(g0 + |g|^2/2)) c_i = c0 prod_m g_m^{alpha_m}/alpha_m! at each
 * centroid, and assembles one stiffness matrix per input term,
 *   K_i[a,b] = sum_T c_i(x_T) |T| grad phi_a . grad phi_b,
 * on one shared CSR pattern (entries whose geometric weight is zero in
 * every element are left out), plus the load F[a] = sum_T |T|/3 (f = 1).
 * Errors: SG_ERR_INVALID_ARG (degenerate or clockwise triangle, bad dof).
 * ---------------------------------------------------------------------- */
int sg_assemble(const sg_basis* b, int n_vert, const double* xy, int n_tri,
                const int32_t* tri, const int32_t* dof, int n,
                const double* g0, const double* g, sg_op** out, void* stream);
int sg_op_info(const sg_op* op, int* n, int* P, int* L_in, int64_t* nnz);
/* device output B [n*P]: the right-hand side b_k = f <Psi_k>, i.e. F in
 * column 0 and zeros elsewhere (Eq. Galerkin_L_exp). */
int sg_op_rhs(const sg_op* op, double* B, void* stream);
/* host outputs: rowptr [n+1], col [nnz], vals [nnz*L_in] (entry-major). */
int sg_op_export(const sg_op* op, int64_t* rowptr, int32_t* col, double* vals);
void sg_destroy_op(sg_op* op);

/* ------------------------------------------------------------------------
 * sg_matvec -- Y = sum_i K_i X G_i, (G_i)_{kj} = m_ijk: the SG operator of
 * Eq. Galerkin_L_exp in the vector-PDE layout (Eqs. linearVecPDE,
 * Ajklinear).  X, Y: device [n*P] FP64, must not alias.  Asynchronous.
 * ---------------------------------------------------------------------- */
int sg_matvec(const sg_op* op, const double* X, double* Y, void* stream);
/* Which kernel family applies the operator (chosen when it is assembled):
 * SG_MV_GENERIC (tiled, any basis with L_in <= 32 and P <= 64), SG_MV_WIDE
 * (one wave per row: L_in > 32 or P > 64), SG_MV_PAIR (fixed basis, two
 * lanes per row), SG_MV_STAGED (fixed basis, input terms split between
 * waves, neighbour rows staged in LDS; needs rows whose neighbours form a
 * few runs of consecutive rows per block of 128), SG_MV_GROUPED (a wide
 * fixed basis, M = 6, p_in = 2, p = 3: input terms and output modes split
 * between the waves of a 64-row tile, neighbour rows staged in LDS).
 * Host call. */
enum { SG_MV_GENERIC = 0, SG_MV_WIDE = 1, SG_MV_PAIR = 2, SG_MV_STAGED = 3, SG_MV_GROUPED = 4,
       SG_MV_MATRIX_FREE = 5, SG_MV_ROW_TILED = 6 };
int sg_matvec_kernel(const sg_op* op, int* kind);
/* sg_matvec_row_tiled -- switch the row-tiled kernel of a wide operator on
 * (enable != 0, the default where it is built) or off (the one-wave-per-row
 * kernel SG_MV_WIDE).  The same operator, Y = sum_i K_i X G_i (Eq.
 * Galerkin_L_exp), with one lane per row over tiles of 64 rows.  It is
 * built for input bases with L > 32 terms and P <= 48 output modes, on
 * patterns of at most 7 entries per row whose neighbour rows form at most 4
 * runs of at most 256 rows per tile (lattice-ordered P1 meshes), e.g. the
 * Jacobian and secant operators of sg_nl_setup (the handles that
 * sg_nl_jac_op and sg_nl_mean_op return may be passed, cast from const);
 * SG_ERR_UNSUPPORTED when enabling an operator without it.  Cached graphs of
 * the operator are dropped on a change.  Host call. */
int sg_matvec_row_tiled(sg_op* op, int enable);
/* sg_matvec_matrix_free -- apply the operator without reading its stored
 * values (the matrix-free approach the paper names as future work, Sec. 5):
 * each row forms its K_i[a, b] from the six elements around it, with the
 * input coefficients c_i(T) = c0(T) prod_m g_m(T)^alpha_m / alpha_m!
 * regenerated from the element's fields (Eq. inputlogn) and the element's
 * local stiffness |T| grad phi_a . grad phi_b (two matrices for a uniform
 * lattice, else one per element), then contracts as the staged kernel does.
 * Needs a mesh that is the structured N x N lattice of "/"-cut squares
 * (vertices may be moved) in the lattice numbering (element 2(jN+i) =
 * (v(i,j), v(i+1,j), v(i+1,j+1)), 2(jN+i)+1 = (v(i,j), v(i+1,j+1), v(i,j+1)),
 * v(i,j) = j(N+1)+i, unknowns numbered x-fastest), a basis with the staged
 * kernel (SG_MV_STAGED) and input order <= 2; else SG_ERR_UNSUPPORTED.
 * enable = 0 returns to the stored values.  Results equal the stored-value
 * apply up to rounding.  Synchronous; drops captured graphs that use the op. */
int sg_matvec_matrix_free(sg_op* op, int enable, void* stream);
/* Work-group shape of the staged kernel: 1, 2 or 4 tiles of 64 rows per
 * work-group (2 after assembly when it fits).  sg_matvec_autotune times
 * `reps` launches of every shape that fits (HIP events on `stream`, on an
 * internal zero input), keeps the fastest and writes ms_out[3] (ms per
 * launch for 1, 2, 4 tiles; -1 where a shape does not fit); synchronous.
 * sg_matvec_select sets a shape directly (e.g. a cached tuning result);
 * sg_matvec_tiles reads it (0 for the other kernel families).  Both return
 * SG_ERR_UNSUPPORTED for operators without the staged kernel or a shape
 * that does not fit.  A new shape drops the captured Arnoldi-step graphs of
 * the operator.  Not to be called while the operator is in use. */
int sg_matvec_autotune(sg_op* op, int reps, double* ms_out, void* stream);
int sg_matvec_select(sg_op* op, int tiles);
int sg_matvec_tiles(const sg_op* op, int* tiles);

/* ------------------------------------------------------------------------
 * ras_setup / ras_apply -- one-level restricted additive Schwarz, Eq. RASsto:
 *   Z = sum_s R_s^T D_s (R_s K_0 R_s^T)^{-1} (R_s R) G_0^{-1}
 * owner [n] (host): subdomain of every unknown (0..n_sub-1, D_s = owned).
 * Subdomain s grows by `overlap` layers of mesh-graph neighbours.  The local
 * solve is mean-based (K_0 and G_0 = diag(alpha!)), exact up to rounding:
 * each local matrix is factored on the device as a block-tridiagonal matrix
 * (consecutive blocks of a breadth-first ordering), keeping the inverse of
 * every Schur complement in `prec` (FP64, FP32 or BF16; the block products
 * run on the matrix cores, FP32 accumulation for the low precisions).
 * Blocks wider than 64 nodes give SG_ERR_UNSUPPORTED; a non-positive pivot
 * gives SG_ERR_NUMERIC.
 * ras_apply: R, Z device [n*P] FP64, must not alias.  Asynchronous.
 * ---------------------------------------------------------------------- */
int ras_setup(const sg_op* op, const int32_t* owner, int n_sub, int overlap,
              sg_prec prec, sg_ras** out, void* stream);
/* Refactor with the current values of op, which must have the pattern the
 * ras was built for (e.g. the same op after its values changed, as in each
 * Newton step).  Synchronous.  Errors: SG_ERR_INVALID_ARG on a pattern
 * mismatch, SG_ERR_NUMERIC on a non-positive pivot. */
int ras_refactor(sg_ras* r, const sg_op* op, void* stream);
/* Apply path.  Sweep (default): the block-tridiagonal forward/backward
 * sweeps with the stored Schur-complement inverses.  Dense: the rows of the
 * owned nodes of each local inverse, (R_s K_0 R_s^T)^{-1} restricted to
 * D_s, formed once by the sweeps on identity blocks (FP64) and stored in the
 * ras precision; an apply is then one matrix-core product per subdomain
 * (owned rows x local nodes times local nodes x P), whose bytes scale with
 * the precision.  Both compute the same operator (up to rounding).
 * ras_select: 0 = sweep, 1 = dense with 64 owned rows per wave, 2 = dense
 *   with 32, 3 = fused dense: one work-group per subdomain gathers its
 *   right-hand sides into on-chip memory itself, in chunks of about a
 *   seventh of its local nodes held in a ring of two, and streams the rows
 *   once (available where two chunks of P_pad columns plus n_local node ids
 *   fit one work-group's LDS and P <= 48, FP64: P <= 16; else
 *   SG_ERR_UNSUPPORTED).  With Kronecker local solves the fused path mixes
 *   its output by Gt^{-1} instead of the right-hand side by Gt^{-1} G_0.
 *   The dense rows are built on first use; device memory
 *   sum_s ceil16(n_own(s)) * ceil64(n_local(s)) entries.  Synchronous.
 * ras_autotune: builds the dense rows if needed, times `reps` applies of
 *   each of the four with HIP events on `stream` (internal zero input),
 *   keeps the fastest; ms (host [4], may be NULL): in the order above,
 *   -1 for a path that is not available.  Synchronous.
 * ras_path_info: current path (as for ras_select) and the bytes of the
 *   dense rows (0 if not built).  A refactorisation rebuilds the dense rows.
 * A new path drops the captured Arnoldi-step graphs that use the handle. */
int ras_select(sg_ras* r, int dense, void* stream);
int ras_autotune(sg_ras* r, int reps, double* ms, void* stream);
int ras_path_info(const sg_ras* r, int* dense, int64_t* dense_bytes);
/* host outputs (any may be NULL): number of local nodes per subdomain
 * [n_sub], number of level sets per subdomain [n_sub], and the total bytes
 * of stored Schur-complement inverses. */
int ras_info(const sg_ras* r, int32_t* n_local, int32_t* n_levels, int64_t* factor_bytes);
/* ras_set_local -- the local solve of every subdomain (Sec. 3 uses the full
 * local SG block; the Kronecker-product preconditioners it cites for SG
 * systems motivate the second kind).  SG_LOCAL_MEAN (the default) solves with
 * K_0 (x) G_0.  SG_LOCAL_KRON solves with K_0 (x) Gt, Ullmann's Kronecker
 * factor Gt = sum_i (<K_i, K_0>_F / <K_0, K_0>_F) G_i, the G that minimises
 * ||sum_i K_i (x) G_i - K_0 (x) G||_F, computed from `op`'s values (the
 * global stiffness matrices, stored pattern).  Applied as a per-node mixing of
 * the right-hand side by Gt^{-1} G_0 (a [n*P] FP64 buffer the handle
 * allocates) before the unchanged mean-based kernels, since the mixing
 * commutes with restriction, local K_0 solve and partition of unity; every
 * path and precision takes it, and ras_refactor recomputes Gt.  Synchronous;
 * captured Arnoldi-step graphs that use the handle are dropped.
 * SG_ERR_NUMERIC if Gt is singular. */
int ras_set_local(sg_ras* r, const sg_op* op, sg_local_kind mode, void* stream);
/* host output: Gt [P*P] row-major, for SG_LOCAL_KRON handles. */
int ras_local_factor(const sg_ras* r, double* gt);
int ras_apply(const sg_ras* r, const double* R, double* Z, void* stream);
void sg_destroy_ras(sg_ras* r);

/* ------------------------------------------------------------------------
 * amg_setup / amg_vcycle -- the coarse problem of the two-grid cycle
 * (Eq. coarse, A_c = R_0 A R_0^T) with the Nicolaides coarse space
 * Z_s = R_s^T D_s 1 of the subdomains of `ras`, so that
 *   A_c = sum_i (Z^T K_i Z) (x) G_i      (coarse vectors [n_sub*P]).
 * kind SG_COARSE_MEAN_EXACT: x_c = (C_0 (x) G_0)^{-1} b_c, exact.
 * kind SG_COARSE_AMG: one V(1,1) cycle of smoothed aggregation on A_c
 * (strength theta = 0.08 on the mean-mode entries, three-pass greedy
 * aggregation, prolongator smoothing with omega = (4/3)/rho(D^{-1}A),
 * <= 4 levels / <= 8 block-nodes, damped block-Jacobi omega_s = 2/3 whose
 * block inverses are stored in `prec`, coarsest level exact in FP64).
 * For an operator from sg_assemble the handle also holds (A Z) on the rows
 * where it is non-zero (next to a subdomain interface or the boundary), so
 * that the two-grid cycle forms r - A z2 as (r - A z1) - (A Z) e_c instead
 * of a matvec; the cycle writes a buffer of the handle (P doubles per
 * (row, subdomain) entry of A Z), so cycles that share a handle must be
 * ordered on one stream.  b_c, x_c: device [n_sub*P] FP64.  Asynchronous.
 * ---------------------------------------------------------------------- */
int amg_setup(const sg_op* op, const sg_ras* ras, sg_coarse_kind kind, sg_prec prec,
              sg_amg** out, void* stream);
/* host outputs: number of levels, and block-nodes per level [4]; agg, if
 * not NULL, receives the first-level aggregate of every subdomain [n_sub]
 * (-1 when there is a single level). */
int amg_info(const sg_amg* a, int* n_levels, int32_t* nodes_per_level, int32_t* agg);
/* host outputs (any may be NULL): the P x P FP64 blocks stored for level
 * `level` (0 .. n_levels-1) of an SG_COARSE_AMG hierarchy: its operator,
 * prolongator and restriction; on the coarsest level the operator is the
 * dense inverse (n_l^2 blocks) and the other two are 0.  For sizing the
 * bytes a V-cycle moves.  SG_ERR_INVALID_ARG for a level out of range. */
int amg_level_blocks(const sg_amg* a, int level, int64_t* a_blocks, int64_t* p_blocks,
                     int64_t* r_blocks);
/* The kind's own coarse solve: one V-cycle (SG_COARSE_AMG) or the exact
 * mean-based solve, whatever amg_set_inner chose. */
int amg_vcycle(const sg_amg* a, const double* b_c, double* x_c, void* stream);
/* amg_set_inner -- the coarse solve of the two-grid cycle becomes GMRES on
 * A_c (Sec. 3, the 2GV2 / 2GV3 variants), flexible, no restart, classical
 * Gram-Schmidt with a second pass, stopped at ||b_c - A_c x_c|| <= rtol ||b_c||
 * (the Givens estimate) or after max_its steps (1..200), from x_c = 0.
 * SG_INNER_GMRES_AMG preconditions each step with one V-cycle (the paper
 * uses BoomerAMG, rtol 1e-5); SG_INNER_GMRES_BJ with the block Jacobi of
 * A_c's diagonal P x P blocks held in the hierarchy's precision, i.e. a
 * one-level Schwarz method without overlap whose subdomains are single
 * coarse nodes (the paper uses one-level RAS, rtol 1e-2, <= 100 steps).
 * SG_INNER_NONE restores the V-cycle.  Needs kind SG_COARSE_AMG; a
 * hierarchy of one level is already an exact solve and keeps it.  Allocates
 * the inner basis ((2 max_its + 2) n_sub P doubles) and a pinned host slot;
 * a call that changes max_its first waits for the device.
 * The inner solve reads its residual estimate on the host after every step,
 * so it synchronises the stream: fgmres_solve does not capture graphs of
 * Arnoldi steps while it is active, and a caller must not capture it. */
int amg_set_inner(sg_amg* a, sg_inner_kind inner, double rtol, int max_its);
/* host outputs (any may be NULL): inner solves so far, their total steps,
 * and the steps of the last one. */
int amg_inner_stats(const sg_amg* a, int64_t* calls, int64_t* its, int* last_its);
/* The coarse solve the two-grid cycle uses: amg_vcycle, or the inner GMRES
 * of amg_set_inner (then synchronous).  b_c, x_c device [n_sub*P], no alias. */
int amg_coarse_solve(const sg_amg* a, const double* b_c, double* x_c, void* stream);
/* ------------------------------------------------------------------------
 * amg_setup_geometric -- the coarse space of Eq. coarse (Sec. 3) taken from
 * a coarser triangulation, as in the fine:coarse ratio study of Sec. 5 (the
 * ratio_deter / ratio_stoc tables): R_0^T = P_0 interpolates the P1 functions
 * of the N/ratio x N/ratio lattice (the same "/"-cut squares) at the fine
 * nodes, and
 *   A_c = P_0^T A P_0 = sum_i (P_0^T K_i P_0) (x) G_i   ((N/ratio - 1)^2 * P).
 * op must come from sg_assemble on the structured N x N lattice (jittered
 * vertices allowed: P_0 is defined on the lattice topology), ratio >= 1
 * dividing N with N/ratio >= 2.  Fine node (i, j) lies in coarse cell
 * (i / r, j / r) at (a, b) = ((i mod r)/r, (j mod r)/r); its weights are
 * (1-a, a-b, b) on the corners (0,0), (1,0), (1,1) when a >= b, else
 * (1-b, a, b-a) on (0,0), (1,1), (0,1); boundary coarse nodes are dropped.
 * A_c is formed on the host from op's values (exact cancellations, such as
 * the hypotenuse pairs of a right-angled lattice, are left out of its
 * pattern).  The coarse solve is FGMRES on A_c (Sec. 3: GMRES for the coarse
 * grid) from x_c = 0, classical Gram-Schmidt with the conditional second
 * pass, restart min(max_its, 64), stopped at ||b_c - A_c x_c|| <= rtol ||b_c||
 * or after max_its steps (rtol in (0, 1), max_its 1..1000), right-
 * preconditioned by the two-grid cycle of the coarse problem itself: RAS on
 * owner_c [(N/ratio - 1)^2] (host; n_sub_c subdomains, `overlap` layers of
 * coarse-lattice neighbours, local solves in `prec`) with its own damping
 * (estimated here) and, unless level_coarse is SG_COARSE_NONE (one-level, the
 * 2GV2 reading), the Nicolaides coarse correction of kind level_coarse
 * (SG_COARSE_MEAN_EXACT or SG_COARSE_AMG).  The handle serves wherever an
 * sg_amg does (sg_precond_apply, fgmres_solve, amg_coarse_solve,
 * sg_coarse_restrict / sg_coarse_prolong_add on [(N/ratio - 1)^2 * P]
 * coarse vectors) with any RAS of op; its coarse solve synchronises the
 * stream, so the Arnoldi steps of a solve that uses the handle are not
 * captured into graphs, while the coarse FGMRES replays its own steps as
 * graphs captured on first use; amg_inner_stats counts its steps.
 * Synchronous.  Errors:
 * SG_ERR_INVALID_ARG (not a lattice operator, bad ratio or arguments),
 * and those of ras_setup / amg_setup on the coarse problem.
 * ---------------------------------------------------------------------- */
int amg_setup_geometric(const sg_op* op, int ratio, const int32_t* owner_c, int n_sub_c,
                        int overlap, sg_coarse_kind level_coarse, sg_prec prec, double rtol,
                        int max_its, sg_amg** out, void* stream);
/* host outputs (any may be NULL): coarse unknowns (N/ratio - 1)^2, entries of
 * the coarse pattern, and the coarse smoother's damping.  SG_ERR_INVALID_ARG
 * for other kinds. */
int amg_geometric_info(const sg_amg* a, int* n_c, int64_t* nnz_c, double* omega_c);
/* The coarse operator A_c of a geometric handle (owned by it, valid until
 * sg_destroy_amg), e.g. for sg_op_export; NULL for other kinds. */
const sg_op* amg_geometric_op(const sg_amg* a);

/* r_c = Z^T R (sum over owned nodes) and Y += Z e_c.  Asynchronous. */
int sg_coarse_restrict(const sg_amg* a, const double* R, double* r_c, void* stream);
int sg_coarse_prolong_add(const sg_amg* a, const double* e_c, double* Y, void* stream);
void sg_destroy_amg(sg_amg* a);

/* ------------------------------------------------------------------------
 * Two-grid preconditioner, Eq. RAS_2L read as the cycle the text describes
 * (the printed Q P Q^{-1} term equals P^T):
 *   z1 = w M r,  z2 = z1 + Q (r - A z1),  z = z2 + w M (r - A z2),
 * M = ras, Q = Z (coarse solve of `amg`) Z^T, w = the smoother damping;
 * r - A z2 is (r - A z1) - (A Z) e_c where `amg` holds A Z for `op`.
 * amg may be NULL (one-level: z = w M r).  ws: device workspace of at
 * least sg_precond_workspace_bytes(op, amg).  R, Z device [n*P], no alias.
 * ---------------------------------------------------------------------- */
size_t sg_precond_workspace_bytes(const sg_op* op, const sg_amg* amg);
int sg_precond_apply(const sg_op* op, const sg_ras* ras, const sg_amg* amg, double omega,
                     const double* R, double* Z, void* ws, size_t ws_bytes, void* stream);
/* sg_precond_apply_noalloc -- the two-grid cycle of sg_precond_apply for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the workspace comes from a
 * static device array of SG_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends, instead of a `ws` argument.  Same arguments and result as
 * sg_precond_apply; the call makes no device allocation.  All calls on one
 * GPU share that GPU's scratch, so calls that overlap on one GPU (other
 * streams, other threads) race; order them on one stream.  The scratch keeps
 * the last call's contents; the cycle writes every entry before reading it.
 * Errors: SG_ERR_WORKSPACE when sg_precond_workspace_bytes(op, amg) exceeds
 * SG_NOALLOC_SCRATCH_BYTES (amg == NULL needs none); as sg_precond_apply
 * otherwise.  With an inner coarse GMRES (amg_set_inner) the call
 * synchronises the stream, as the apply with a workspace does. */
#define SG_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int sg_precond_apply_noalloc(const sg_op* op, const sg_ras* ras, const sg_amg* amg,
                             double omega, const double* R, double* Z, void* stream);
/* Damping of the smoother: rho = power estimate of rho(M A) (`its`
 * iterations from a SplitMix64 field: entry i of the flattened [n*P] start
 * is output i + 1 from state 0, top 53 bits mapped to [-1/2, 1/2));
 * omega = min(1, 1.8/rho).  Synchronous. */
int sg_smoother_damping(const sg_op* op, const sg_ras* ras, int its, double* rho,
                        double* omega, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * fgmres_solve -- right-preconditioned flexible GMRES(m) (the outer solver
 * of Secs. 3-4) in FP64: Gram-Schmidt Arnoldi (opts->ortho), Givens rotations,
 * stopping test |g_{j+1}| <= rtol ||b|| (relative to the right-hand side),
 * confirmed by the true residual ||b - A x||; restart from x otherwise.
 * x holds the initial guess on entry and the solution on return (device).
 * ras/amg may be NULL (no preconditioner / one-level).  ws: device
 * workspace of at least fgmres_workspace_bytes(op, amg, restart), 256-byte
 * aligned (SG_ERR_INVALID_ARG otherwise).
 * Returns SG_OK, SG_NOT_CONVERGED (max_it reached) or an error.
 * Synchronous; the host reads one residual estimate per iteration.
 * With use_graph, step j (preconditioner cycle, matvec, the j+1 Gram-Schmidt
 * kernels, normalisation and Givens update) is captured on a library stream
 * the first time it runs and replayed on `stream` afterwards; the graph only
 * references the handles' memory and ws, and is dropped when a handle it
 * references is destroyed (sg_graph_cache_clear drops all).
 * ---------------------------------------------------------------------- */
typedef enum {
    SG_ORTHO_MGS = 0,       /* modified Gram-Schmidt                         */
    SG_ORTHO_CGS_DGKS = 1,  /* classical, second pass when ||w|| drops by    */
                            /* more than 1 - 1/sqrt(2) (Daniel-Gragg-Kaufman-  */
                            /* Stewart)                                       */
    SG_ORTHO_CGS = 2,       /* classical, one pass                           */
    SG_ORTHO_CGS_BLOCK2 = 3,/* classical, one pass over the basis for a      */
                            /* block of 2 directions: the block at column j  */
                            /* takes u_1 = A M v_j, u_{t+1} = A M u_t (the   */
                            /* flexible direction of column j+t is M u_t),   */
                            /* projects all against v_0..v_j together, then  */
                            /* orthonormalises them by a Cholesky factor of  */
                            /* their Gram matrix (repeated once where a      */
                            /* pivot keeps less than 1e-4 of its column's    */
                            /* norm).  Same Krylov space as one step at a    */
                            /* time for a fixed linear preconditioner; the   */
                            /* basis is read once per block.  Convergence is */
                            /* checked after every block; the blocks shrink  */
                            /* to fit the restart length and the step budget.*/
    SG_ORTHO_CGS_BLOCK3 = 4,/* the same with blocks of 3 directions          */
    SG_ORTHO_CGS_BLOCK4 = 5 /* the same with blocks of 4 directions          */
} sg_ortho;

typedef struct {
    int restart;        /* m (>= 1)                                   */
    int max_it;         /* total Arnoldi steps allowed                */
    double rtol;        /* relative to ||b||                          */
    double omega;       /* smoother damping (<= 0: estimate it)       */
    int use_graph;      /* 1: replay each Arnoldi step as a captured  */
                        /*    HIP graph (captured once per handles,   */
                        /*    workspace, m, omega and step index)     */
    int ortho;          /* sg_ortho: Arnoldi orthogonalisation         */
} sg_krylov_opts;

typedef struct {
    int iterations;
    int restarts;
    int converged;
    double true_relres;      /* ||b - A x|| / ||b|| at return          */
    double omega;            /* damping used                           */
    double ms_solve;         /* wall time of the Krylov loop            */
    double* history;         /* host, may be NULL: estimate / ||b||     */
    int history_cap;         /* entries available in history            */
    int history_len;         /* entries written                         */
} sg_krylov_stats;

size_t fgmres_workspace_bytes(const sg_op* op, const sg_amg* amg, int restart);
/* Drop every cached Arnoldi-step graph (e.g. before freeing a workspace that
 * was used with use_graph).  Returns the number of graphs released. */
int sg_graph_cache_clear(void);
int fgmres_solve(const sg_op* op, const sg_ras* ras, const sg_amg* amg,
                 const double* b, double* x, const sg_krylov_opts* opts,
                 sg_krylov_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Nonlinear problem and Newton's method.
 *
 * The paper's nonlinear model -div(c(x,xi) q(u) grad u) = f (Eq.
 * NLP_StrongPDE, Galerkin system Eqs. stonlp_system / vectorvalPDENL, which
 * the paper linearises by Picard iterations) with q(u) = kappa(u) =
 * 1 + a1 u + a2 u^2 (the paper's 1 + alpha u: a1 = alpha, a2 = 0), f = 1 and
 * homogeneous Dirichlet data, solved by inexact Newton with backtracking or
 * by Picard iterations (newton_solve).  The residual is R(U) = F e_0 - A(U) with
 *   A(U)[a, m] = sum_T |T| E[c_T kappa(u_T) (grad u_T . grad phi_a) Psi_m],
 * c_T the input PCE (first L_in terms) at the centroid of T and u_T the
 * centroid value of u.  All expectations are exact (up to rounding): the
 * library forms the chaos coefficients of degree <= 2p of c_T kappa(u_T)
 * and c_T kappa'(u_T) (grad u_T . grad phi_a) by chaos products, so the
 * Jacobian dA/dU is the Kronecker sum sum_gamma K_gamma (x) T_gamma with
 * L2 = (M+2p)!/(M! (2p)!) terms on the unpruned P1 pattern.
 *
 * sg_nl_setup -- element geometry, input PCE, product tables and both
 *   operators (the Picard part K1 and the Jacobian K1 + K2) for the basis b
 *   (its M, p_in, p) on the mesh (same arguments as sg_assemble).
 *   a1 finite, a2 >= 0.  Synchronous.  Errors: SG_ERR_INVALID_ARG.
 * sg_nl_eval -- assemble K1 and the Jacobian at U (device, [n x P]) and, if
 *   R is not NULL, write R(U) (device, [n x P]).  Asynchronous.
 * sg_nl_jac_apply -- Y = J X with the Jacobian of the last sg_nl_eval.
 * sg_nl_export -- host copies of the pattern (rowptr [n+1], col [nnz]) and
 *   of the values of K1 and of the Jacobian ([nnz x L2], entry-major,
 *   gamma-th value = coefficient of T_gamma); any pointer may be NULL.
 * sg_nl_mean_op / sg_nl_jac_op -- the K1 and Jacobian operators as sg_op
 *   handles owned by the sg_nl (for ras_setup: K1's gamma = 0 term is the
 *   mean-coefficient stiffness used by the RAS local solves; for
 *   amg_setup / sg_precond_apply / fgmres_solve: the Jacobian).
 * ---------------------------------------------------------------------- */
typedef struct sg_nl sg_nl;

int sg_nl_setup(const sg_basis* b, int n_vert, const double* xy, int n_tri,
                const int32_t* tri, const int32_t* dof, int n, const double* g0,
                const double* g, double a1, double a2, sg_nl** out, void* stream);
int sg_nl_info(const sg_nl* nl, int* n, int* P, int* L2, int64_t* nnz);
int sg_nl_eval(sg_nl* nl, const double* U, double* R, void* stream);
int sg_nl_jac_apply(const sg_nl* nl, const double* X, double* Y, void* stream);
int sg_nl_export(const sg_nl* nl, int64_t* rowptr, int32_t* col, double* k1, double* jac);
const sg_op* sg_nl_mean_op(const sg_nl* nl);
const sg_op* sg_nl_jac_op(const sg_nl* nl);
/* New input coefficient fields (g0 [n_tri], g [M][n_tri], host) on the same
 * mesh and basis: only the element coefficients are recomputed.  Synchronous. */
int sg_nl_set_coefficients(sg_nl* nl, const double* g0, const double* g, void* stream);
void sg_destroy_nl(sg_nl* nl);

/* ------------------------------------------------------------------------
 * newton_solve -- inexact Newton (method SG_NEWTON) or Picard iterations
 * (SG_PICARD) on R(U) = 0 from the initial guess in U
 * (device, [n x P], overwritten by the last iterate).  Step k:
 *   eta_k = max(1e-12, min(eta_max, ||R_k|| / ||F||));
 *   RAS on K1 (mean-coefficient local solves, subdomains `owner`, overlap)
 *   refactored, and the coarse solver `coarse` on the Jacobian built at the
 *   first step and rebuilt every amg_rebuild steps after it (0: never: the
 *   coarse problem of the first Jacobian is kept, a lagged preconditioner);
 *   FGMRES(restart) solves J d = R_k to relative tolerance eta_k from d = 0;
 *   lambda = 1, halved (at most 9 times) until
 *   ||R(U + lambda d)|| <= (1 - 1e-4 lambda) ||R_k||, the last trial taken
 *   otherwise;  U += lambda d.
 * The forcing term is safeguarded against over-solving the last steps:
 * eta_k = min(eta_max, max(eta_k, 0.5 tol ||F|| / ||R_k||)).
 * SG_PICARD: the same with the secant operator K1(U) (A(U) = K1(U) U) in place
 * of the Jacobian, for FGMRES and the coarse solver, and the full step
 * lambda = 1 (U_{k+1} = K1(U_k)^{-1} F e_0 up to the inner tolerance).
 * Stops when ||R|| / ||F|| <= tol (||F|| = norm of F e_0) or, if du_tol > 0,
 * when ||lambda d|| <= du_tol ||U|| (the paper's Picard criterion).  ws: device
 * workspace of newton_workspace_bytes(nl, n_sub, coarse, restart) bytes,
 * 256-byte aligned.
 * Returns SG_OK, SG_NOT_CONVERGED (max_steps reached) or an error.
 * Synchronous.
 * ---------------------------------------------------------------------- */
typedef struct {
    int max_steps;
    double tol;          /* on ||R|| / ||F||                             */
    double eta_max;      /* cap of the inner relative tolerance (0,1)    */
    int restart;         /* FGMRES restart length                       */
    int max_it;          /* Arnoldi steps per linear solve              */
    double omega;        /* smoother damping (<= 0: estimate per step)  */
    int use_graph;       /* as in sg_krylov_opts                        */
    int ortho;           /* as in sg_krylov_opts                        */
    int amg_rebuild;     /* coarse-solver rebuild interval in steps (>= 0) */
    int method;          /* SG_NEWTON or SG_PICARD                       */
    double du_tol;       /* stop on ||lambda d|| <= du_tol ||U|| (0: off) */
    int ras_path;        /* RAS apply path, kept through the refactorisations:
                            0 sweep, 1..3 as in ras_select, -1 the fastest
                            of ras_autotune at the first step            */
} sg_newton_opts;

enum { SG_NEWTON = 0, SG_PICARD = 1 };

typedef struct {
    int steps;
    int krylov_its;          /* total Arnoldi steps                       */
    int converged;
    double relres;           /* ||R|| / ||F|| at return                   */
    double last_lambda;
    double last_du;          /* ||lambda d|| / ||U|| of the last step (if du_tol > 0) */
    double ms_total, ms_eval, ms_setup, ms_krylov;
    double* history;         /* host, may be NULL: ||R_k|| / ||F||, k = 0..steps */
    int* krylov_its_per_step;/* host, may be NULL: entry k-1 for step k   */
    int history_cap;
    int history_len;
} sg_newton_stats;

size_t newton_workspace_bytes(const sg_nl* nl, int n_sub, sg_coarse_kind coarse, int restart);
int newton_solve(sg_nl* nl, const int32_t* owner, int n_sub, int overlap, sg_prec prec,
                 sg_coarse_kind coarse, double* U, const sg_newton_opts* opts,
                 sg_newton_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * newton_guess -- initial guess for newton_solve from a predicted field
 * U_pred (device [n x P], e.g. the output of nn_forward).  Three damped
 * Jacobi sweeps (omega 0.6, the mean-coefficient diagonal K1_0[a,a] k!)
 * smooth U_pred into U_s; with W_d its part on the chaos modes of total
 * degree d (d = 0..p), one Gauss-Newton step restricted to span{W_d} gives
 * U_proj = sum_d (1 + beta_d) W_d, beta minimising
 * ||R(U_s) - J(U_s) sum_d beta_d W_d||; the better of U_s and U_proj is
 * the smoothed candidate.  U0 (device) receives the candidate with the
 * smallest residual among the zero guess, U_pred and the smoothed one, so
 * Newton never starts from a larger residual than with the zero guess.
 * relres (host [3], may be NULL): ||R|| / ||F|| of the three candidates;
 * choice: 0 = zero, 1 = prediction, 2 = smoothed.
 * ws: newton_guess_workspace_bytes(nl) bytes of device memory.  Synchronous.
 * ---------------------------------------------------------------------- */
size_t newton_guess_workspace_bytes(const sg_nl* nl);
int newton_guess(sg_nl* nl, const double* U_pred, double* U0, double* relres, int* choice,
                 void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Learned predictor: a convolutional network on a W x H vertex grid (the
 * project's own design; the paper has no learned component).  NHWC layout
 * (sample, y, x, channel).  n_layers 3x3 convolutions with zero padding,
 * channels[0] -> channels[1] -> ... -> channels[n_layers] (each <= 64), ReLU
 * between layers:
 *   Z_l = conv3x3(A_{l-1}, W_l) + b_l,  A_l = max(Z_l, 0),  O = Z_L,
 *   U[s, y, x, k] = env[y, x] * oscale[k] * O[s, y, x, k].
 * Convolutions run on the matrix cores with BF16 operands and FP32
 * accumulation; weights are FP32 master copies updated by Adam.
 * Parameters are one FP32 vector: W_1 [3][3][c_0][c_1], b_1 [c_1], W_2, ...
 * (C order).  The loss of nn_loss_grad is mean (env O - T / oscale)^2 over
 * all samples, pixels and the c_L output channels.
 * nn_create: device buffers for up to max_batch samples; parameters zero.
 * nn_set_params: host FP32 parameters, resets the Adam state.
 * nn_get_params: host copies of the parameters and of the last gradient
 *   (either may be NULL).
 * nn_set_output_map: host env [H*W] and oscale [c_L].
 * nn_forward: X device FP64 [B,H,W,c_0] -> U device FP64 [B,H,W,c_L].
 * nn_loss_grad: X and T (device FP64 [B,H,W,c_L]) -> loss (host) and the
 *   gradient kept for nn_adam_step.  Synchronous.
 * nn_adam_step: one Adam update (bias-corrected) with the last gradient.
 * ---------------------------------------------------------------------- */
typedef struct sg_nn sg_nn;
int nn_create(int n_layers, const int32_t* channels, int H, int W, int max_batch, sg_nn** out);
int64_t nn_param_count(const sg_nn* nn);
int nn_set_params(sg_nn* nn, const float* params);
int nn_get_params(const sg_nn* nn, float* params, float* grads);
int nn_set_output_map(sg_nn* nn, const float* env, const float* oscale);
/* nn_fit_output_map: the output map from data, on the device: env = shape /
 * max(shape) (shape: device FP64 [H*W], e.g. the solution of the problem with
 * unit coefficient, which vanishes where every chaos mode does) and
 * oscale[k] = max(RMS over the B samples and all pixels of T[.., k], 1e-30) /
 * RMS(env) (T: device FP64 [B,H,W,c_L], training targets).  Synchronous. */
int nn_fit_output_map(sg_nn* nn, const double* shape, const double* T, int B, void* stream);
/* nn_input_fields: the network's input channels at npts points (device FP64):
 * X[p] = [c0, g_1 .. g_M] with c0 = exp(g0 + |g|^2 / 2), the mean of the
 * log-normal coefficient (Eq. inputlogn); g0 [npts], g [M][npts] (row m
 * contiguous), X [npts][M+1].  M <= 16.  Asynchronous. */
int nn_input_fields(int npts, int M, const double* g0, const double* g, double* X, void* stream);
int nn_forward(sg_nn* nn, const double* X, int B, double* U, void* stream);
int nn_loss_grad(sg_nn* nn, const double* X, const double* T, int B, double* loss, void* stream);
int nn_adam_step(sg_nn* nn, float lr, float beta1, float beta2, float eps, void* stream);
void nn_destroy(sg_nn* nn);

#ifdef __cplusplus
}
#endif
#endif /* SGSOLVE_H */
