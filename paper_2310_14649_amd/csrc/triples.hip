// Hermite chaos basis and the triple-product tensor m_ijk = <Psi_i Psi_j Psi_k>
// (Eq. Galerkin_L_exp; only non-zero entries are kept, as the paper states
// for its multiplication tensors).  The multi-index enumeration is
// combinatorial host work; the tensor itself is evaluated on the device from
// the one-dimensional Hermite linearisation coefficients
//   <He_a He_b He_c> = a! b! c! / ((s-a)! (s-b)! (s-c)!),  a+b+c = 2s,
//   s >= max(a,b,c)  (zero otherwise).
#include "common.hpp"

#include <algorithm>
#include <tuple>

namespace sg {

static thread_local std::string g_last_error;

void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

namespace {

constexpr int kMaxM = 8;
constexpr int kMaxOrder = 4;
constexpr int kMaxP = 128;

__device__ double dev_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

__device__ double hermite_triple(int a, int b, int c) {
    int tot = a + b + c;
    if (tot & 1) return 0.0;
    int s = tot >> 1;
    if (s < a || s < b || s < c) return 0.0;
    return dev_fact(a) * dev_fact(b) * dev_fact(c) /
           (dev_fact(s - a) * dev_fact(s - b) * dev_fact(s - c));
}

// One thread per (i, j, k), i < na, j < nb, k < nc (all three index the
// same graded enumeration); dense output [na][nb][nc].
__global__ void triple_dense_kernel(int M, int na, int nb, int nc, const int32_t* __restrict__ alpha,
                                    double* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)na * nb * nc;
    if (idx >= total) return;
    int k = (int)(idx % nc);
    int j = (int)((idx / nc) % nb);
    int i = (int)(idx / ((int64_t)nb * nc));
    double m = 1.0;
    for (int d = 0; d < M && m != 0.0; ++d)
        m *= hermite_triple(alpha[i * M + d], alpha[j * M + d], alpha[k * M + d]);
    out[idx] = m;
}

}  // namespace

// Multi-indices of total degree <= p: by degree, then descending lexicographic.
void enumerate(int M, int p, std::vector<int32_t>& alpha, int& count) {
    alpha.clear();
    count = 0;
    if (M == 0) {
        count = 1;
        return;
    }
    std::vector<int32_t> cur(M);
    for (int d = 0; d <= p; ++d) {
        // recursive descent without recursion: fill slot by slot
        std::vector<int> stack;
        auto rec = [&](auto&& self, int slot, int left) -> void {
            if (slot == M - 1) {
                cur[slot] = left;
                alpha.insert(alpha.end(), cur.begin(), cur.end());
                ++count;
                return;
            }
            for (int v = left; v >= 0; --v) {
                cur[slot] = v;
                self(self, slot + 1, left - v);
            }
        };
        rec(rec, 0, d);
    }
}

int binom(int n, int k) {
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

void sparse_triples(int M, int deg, int na, int nb, int nc, SparseTriples& out) {
    std::vector<int32_t> alpha;
    int cnt = 0;
    enumerate(M, deg, alpha, cnt);
    SG_REQUIRE(na <= cnt && nb <= cnt && nc <= cnt, "triple ranges exceed the degree-%d basis", deg);
    out.a.clear(); out.b.clear(); out.c.clear(); out.v.clear();
    const size_t total = (size_t)na * nb * nc;
    std::vector<double> dense(total, 0.0);
    if (M == 0) {
        dense[0] = 1.0;
    } else {
        DevBuf<int32_t> d_alpha;
        DevBuf<double> d_out(total);
        d_alpha.upload(alpha, nullptr);
        const int threads = 256;
        const int blocks = (int)((total + threads - 1) / threads);
        triple_dense_kernel<<<blocks, threads>>>(M, na, nb, nc, d_alpha.p, d_out.p);
        HIP_LAUNCH_OK();
        d_out.download(dense.data(), total, nullptr);
        HIP_OK(hipDeviceSynchronize());
    }
    for (int k = 0; k < nc; ++k)
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j) {
                const double v = dense[((size_t)i * nb + j) * nc + k];
                if (v != 0.0) {
                    out.a.push_back(i); out.b.push_back(j); out.c.push_back(k); out.v.push_back(v);
                }
            }
}

void upload_triples(const sg_basis& b, TriplesDev& tr, hipStream_t s) {
    tr.P = b.P;
    tr.L = b.L;
    tr.T = b.T;
    std::vector<int32_t> kptr(b.P + 1, 0), tij(b.T);
    for (int t = 0; t < b.T; ++t) {
        kptr[b.tk[t] + 1]++;
        tij[t] = b.ti[t] * b.P + b.tj[t];
    }
    for (int k = 0; k < b.P; ++k) kptr[k + 1] += kptr[k];
    tr.kptr.upload(kptr, s);
    tr.tij.upload(tij, s);
    tr.tval.upload(b.tv, s);
    if (b.L > 32 || b.P > 64) {
        SG_REQUIRE(b.L <= 65536 && b.P <= 128, "wide matvec schedule limits exceeded");
        constexpr int kLanes = 64;
        std::vector<int32_t> lane_ptr(kLanes + 1), slot_ptr(b.P + 1, 0);
        std::vector<uint32_t> sched(b.T);
        int slot = 0;
        for (int c = 0; c < kLanes; ++c) {
            const int t0 = (int)((int64_t)b.T * c / kLanes), t1 = (int)((int64_t)b.T * (c + 1) / kLanes);
            lane_ptr[c] = t0;
            for (int t = t0; t < t1; ++t) {
                const bool flush = (t + 1 == t1) || (b.tk[t + 1] != b.tk[t]);
                sched[t] = (uint32_t)b.ti[t] | ((uint32_t)b.tj[t] << 16) | ((uint32_t)slot << 23) |
                           (flush ? 0x80000000u : 0u);
                if (flush) {
                    slot_ptr[b.tk[t] + 1] = slot + 1;
                    ++slot;
                }
            }
        }
        lane_ptr[kLanes] = b.T;
        SG_REQUIRE(slot <= 256, "wide matvec schedule needs %d slots", slot);
        // every k has at least one triple (i = 0, j = k), so slot_ptr is increasing
        for (int k = 0; k < b.P; ++k)
            SG_REQUIRE(slot_ptr[k + 1] > slot_ptr[k], "output mode %d has no triple", k);
        tr.nslot = slot;
        tr.lane_ptr.upload(lane_ptr, s);
        tr.slot_ptr.upload(slot_ptr, s);
        tr.sched.upload(sched, s);
    }
    HIP_OK(hipStreamSynchronize(s));
}

}  // namespace sg

using namespace sg;

extern "C" {

const char* sg_last_error(void) { return sg::g_last_error.c_str(); }

int sg_version(void) { return 1; }

int sg_build_triples(int M, int p_in, int p_out, sg_basis** out) {
    return guarded([&]() -> int {
        SG_REQUIRE(out != nullptr, "out is NULL");
        SG_REQUIRE(M >= 0 && M <= kMaxM, "M=%d outside [0,%d]", M, kMaxM);
        SG_REQUIRE(p_in >= 0 && p_out >= p_in && p_out <= kMaxOrder,
                   "orders p_in=%d p_out=%d invalid (0 <= p_in <= p_out <= %d)", p_in, p_out,
                   kMaxOrder);
        if (M == 0) {
            SG_REQUIRE(p_in == 0 && p_out == 0, "M=0 requires p_in = p_out = 0");
        }
        int P = binom(M + p_out, p_out);
        int L = binom(M + p_in, p_in);
        SG_REQUIRE(P <= kMaxP, "P=%d exceeds %d", P, kMaxP);
        auto* b = new sg_basis();
        std::unique_ptr<sg_basis> guard(b);
        b->M = M; b->p_in = p_in; b->p = p_out; b->P = P; b->L = L;
        int cnt = 0;
        enumerate(M, p_out, b->alpha, cnt);
        if (cnt != P) SG_THROW(SG_ERR_INVALID_ARG, "internal: enumerated %d of %d", cnt, P);
        b->afact.assign(P, 1.0);
        for (int k = 0; k < P; ++k)
            for (int d = 0; d < M; ++d)
                for (int v = 2; v <= b->alpha[k * M + d]; ++v) b->afact[k] *= v;

        SparseTriples st;
        sparse_triples(M, p_out, L, P, P, st);
        b->ti = std::move(st.a); b->tj = std::move(st.b); b->tk = std::move(st.c);
        b->tv = std::move(st.v);
        b->T = (int)b->tv.size();
        *out = guard.release();
        return SG_OK;
    });
}

int sg_basis_info(const sg_basis* b, int* P, int* L_in, int* n_triples) {
    return guarded([&]() -> int {
        SG_REQUIRE(b != nullptr, "basis is NULL");
        if (P) *P = b->P;
        if (L_in) *L_in = b->L;
        if (n_triples) *n_triples = b->T;
        return SG_OK;
    });
}

int sg_basis_export(const sg_basis* b, int32_t* alpha, int32_t* ijk, double* val) {
    return guarded([&]() -> int {
        SG_REQUIRE(b != nullptr, "basis is NULL");
        if (alpha && !b->alpha.empty())
            std::memcpy(alpha, b->alpha.data(), b->alpha.size() * sizeof(int32_t));
        if (ijk)
            for (int t = 0; t < b->T; ++t) {
                ijk[3 * t] = b->ti[t]; ijk[3 * t + 1] = b->tj[t]; ijk[3 * t + 2] = b->tk[t];
            }
        if (val && b->T) std::memcpy(val, b->tv.data(), b->T * sizeof(double));
        return SG_OK;
    });
}

void sg_destroy_basis(sg_basis* b) { delete b; }

}  // extern "C"
