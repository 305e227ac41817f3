// Compile-time Hermite chaos tables for the specialised SG matvec kernels.
//
// For a fixed number of variables M, input order PIN and output order PO the
// multi-index set (ordered by total degree, then descending lexicographic)
// and the non-zero triple products m_ijk = prod_d <He_{a_d} He_{b_d} He_{c_d}>
// are evaluated by constexpr functions, so that a kernel can unroll the
// contraction  y_k += m_ijk w_ij  with register-resident y and w and the
// coefficients as immediates.  The same values are produced at run time by
// sg_build_triples (triples.hip); the kernel selection checks that the
// basis of the operator matches the table (same P, L_in and triple count).
#pragma once

namespace sg {
namespace tab {

constexpr int cbinom(int n, int k) {
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

constexpr long long cfact(int n) {
    long long f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

constexpr long long he_triple(int a, int b, int c) {
    const int tot = a + b + c;
    if (tot & 1) return 0;
    const int s = tot / 2;
    if (s < a || s < b || s < c) return 0;
    return cfact(a) * cfact(b) * cfact(c) / (cfact(s - a) * cfact(s - b) * cfact(s - c));
}

template <int M, int PO>
struct Basis {
    static constexpr int P = cbinom(M + PO, PO);
    int a[P][M > 0 ? M : 1] = {};
};

// Multi-indices of total degree d in descending lexicographic order are the
// tuples of [0, d]^M with digit sum d, visited from (d,0,..,0) downwards.
template <int M, int PO>
constexpr Basis<M, PO> make_basis() {
    Basis<M, PO> b{};
    int cnt = 0;
    for (int d = 0; d <= PO; ++d) {
        int dig[M > 0 ? M : 1] = {};
        long long total = 1;
        for (int m = 0; m < M; ++m) total *= (d + 1);
        for (long long code = total - 1; code >= 0; --code) {
            long long c = code;
            int sum = 0;
            for (int m = M - 1; m >= 0; --m) {
                dig[m] = (int)(c % (d + 1));
                c /= (d + 1);
                sum += dig[m];
            }
            if (sum == d) {
                for (int m = 0; m < M; ++m) b.a[cnt][m] = dig[m];
                ++cnt;
            }
        }
    }
    return b;
}

template <int M, int PO>
struct BasisHolder {
    static constexpr Basis<M, PO> b = make_basis<M, PO>();
};

template <int M, int PIN, int PO>
constexpr long long triple(const Basis<M, PO>& b, int i, int j, int k) {
    long long m = 1;
    for (int d = 0; d < M && m != 0; ++d) m *= he_triple(b.a[i][d], b.a[j][d], b.a[k][d]);
    return m;
}

template <int M, int PIN, int PO>
constexpr int count_triples() {
    constexpr const auto& b = BasisHolder<M, PO>::b;
    constexpr int P = cbinom(M + PO, PO), L = cbinom(M + PIN, PIN);
    int t = 0;
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < P; ++j)
            for (int k = 0; k < P; ++k)
                if (triple<M, PIN, PO>(b, i, j, k) != 0) ++t;
    return t;
}

template <int M, int PIN, int PO>
struct TripleCount {
    static constexpr int value = count_triples<M, PIN, PO>();
};

template <int M, int PIN, int PO>
struct Table {
    static constexpr int P = cbinom(M + PO, PO);
    static constexpr int L = cbinom(M + PIN, PIN);
    static constexpr int T = TripleCount<M, PIN, PO>::value;
    // sorted by j, then i, then k
    int ti[T] = {}, tj[T] = {}, tk[T] = {};
    double tv[T] = {};
};

template <int M, int PIN, int PO>
constexpr Table<M, PIN, PO> make_table();

template <int M, int PIN, int PO>
struct TableHolder {
    static constexpr Table<M, PIN, PO> t = make_table<M, PIN, PO>();
};

template <int M, int PIN, int PO>
constexpr Table<M, PIN, PO> make_table() {
    Table<M, PIN, PO> t{};
    constexpr const auto& b = BasisHolder<M, PO>::b;
    constexpr int P = Table<M, PIN, PO>::P, L = Table<M, PIN, PO>::L;
    int q = 0;
    for (int j = 0; j < P; ++j)
        for (int i = 0; i < L; ++i)
            for (int k = 0; k < P; ++k) {
                const long long m = triple<M, PIN, PO>(b, i, j, k);
                if (m != 0) {
                    t.ti[q] = i; t.tj[q] = j; t.tk[q] = k; t.tv[q] = (double)m;
                    ++q;
                }
            }
    return t;
}

// Triples of one lane group: the input terms i in [G*LI, G*LI + LI), sorted
// by j, with local index ii = i - G*LI and per-j ranges jptr.
template <int M, int PIN, int PO, int IG, int G>
struct GroupTable {
    static constexpr int P = cbinom(M + PO, PO);
    static constexpr int L = cbinom(M + PIN, PIN);
    static constexpr int LI = (L + IG - 1) / IG;
    static constexpr int count() {
        constexpr const auto& t = TableHolder<M, PIN, PO>::t;
        int c = 0;
        for (int q = 0; q < Table<M, PIN, PO>::T; ++q)
            if (t.ti[q] >= G * LI && t.ti[q] < G * LI + LI) ++c;
        return c;
    }
    static constexpr int T = count();
    int jptr[P + 1] = {};
    int ii[T > 0 ? T : 1] = {}, k[T > 0 ? T : 1] = {};
    double m[T > 0 ? T : 1] = {};
};

template <int M, int PIN, int PO, int IG, int G>
constexpr GroupTable<M, PIN, PO, IG, G> make_group() {
    using GT = GroupTable<M, PIN, PO, IG, G>;
    GT g{};
    constexpr const auto& t = TableHolder<M, PIN, PO>::t;
    int q = 0;
    for (int j = 0; j < GT::P; ++j) {
        g.jptr[j] = q;
        for (int r = 0; r < Table<M, PIN, PO>::T; ++r)
            if (t.tj[r] == j && t.ti[r] >= G * GT::LI && t.ti[r] < G * GT::LI + GT::LI) {
                g.ii[q] = t.ti[r] - G * GT::LI;
                g.k[q] = t.tk[r];
                g.m[q] = t.tv[r];
                ++q;
            }
    }
    g.jptr[GT::P] = q;
    return g;
}

template <int M, int PIN, int PO, int IG, int G>
struct GroupHolder {
    static constexpr GroupTable<M, PIN, PO, IG, G> t = make_group<M, PIN, PO, IG, G>();
};

// Triples of one wave group of the grouped kernel: input terms i in
// [IG*LI, IG*LI + LI) and output modes k in [KG*KL, KG*KL + KL), G = IG +
// IGN*KG, sorted by j, with local indices ii = i - IG*LI and k - KG*KL (field
// k), and per-j ranges jptr.
template <int M, int PIN, int PO, int IGN, int KGN, int G>
struct WaveGroupTable {
    static constexpr int P = cbinom(M + PO, PO);
    static constexpr int L = cbinom(M + PIN, PIN);
    static constexpr int LI = (L + IGN - 1) / IGN;
    static constexpr int KL = (P + KGN - 1) / KGN;
    static constexpr int IG = G % IGN, KG = G / IGN;
    static constexpr bool mine(int i, int k) {
        return i >= IG * LI && i < IG * LI + LI && k >= KG * KL && k < KG * KL + KL;
    }
    static constexpr int count() {
        constexpr const auto& t = TableHolder<M, PIN, PO>::t;
        int c = 0;
        for (int q = 0; q < Table<M, PIN, PO>::T; ++q)
            if (mine(t.ti[q], t.tk[q])) ++c;
        return c;
    }
    static constexpr int T = count();
    int jptr[P + 1] = {};
    int ii[T > 0 ? T : 1] = {}, k[T > 0 ? T : 1] = {};
    double m[T > 0 ? T : 1] = {};
};

template <int M, int PIN, int PO, int IGN, int KGN, int G>
constexpr WaveGroupTable<M, PIN, PO, IGN, KGN, G> make_wave_group() {
    using GT = WaveGroupTable<M, PIN, PO, IGN, KGN, G>;
    GT g{};
    constexpr const auto& t = TableHolder<M, PIN, PO>::t;
    int q = 0;
    for (int j = 0; j < GT::P; ++j) {
        g.jptr[j] = q;
        for (int r = 0; r < Table<M, PIN, PO>::T; ++r)
            if (t.tj[r] == j && GT::mine(t.ti[r], t.tk[r])) {
                g.ii[q] = t.ti[r] - GT::IG * GT::LI;
                g.k[q] = t.tk[r] - GT::KG * GT::KL;
                g.m[q] = t.tv[r];
                ++q;
            }
    }
    g.jptr[GT::P] = q;
    return g;
}

template <int M, int PIN, int PO, int IGN, int KGN, int G>
struct WaveGroupHolder {
    static constexpr WaveGroupTable<M, PIN, PO, IGN, KGN, G> t =
        make_wave_group<M, PIN, PO, IGN, KGN, G>();
};

// Union over the IG = 2 lane groups: entries (j, ii, k) with the triple of
// group 0 (i = ii) and of group 1 (i = LI + ii), either possibly zero, so one
// uniform instruction stream serves both lanes of a row.
template <int M, int PIN, int PO>
struct PairTable {
    static constexpr int P = cbinom(M + PO, PO);
    static constexpr int L = cbinom(M + PIN, PIN);
    static constexpr int LI = (L + 1) / 2;
    static constexpr int count() {
        constexpr const auto& b = BasisHolder<M, PO>::b;
        int c = 0;
        for (int j = 0; j < P; ++j)
            for (int ii = 0; ii < LI; ++ii)
                for (int k = 0; k < P; ++k) {
                    long long m0 = triple<M, PIN, PO>(b, ii, j, k);
                    long long m1 = (LI + ii < L) ? triple<M, PIN, PO>(b, LI + ii, j, k) : 0;
                    if (m0 != 0 || m1 != 0) ++c;
                }
        return c;
    }
    static constexpr int T = count();
    int jptr[P + 1] = {};
    int ii[T] = {}, k[T] = {};
    double m0[T] = {}, m1[T] = {};
};

template <int M, int PIN, int PO>
constexpr PairTable<M, PIN, PO> make_pair_table() {
    using PT = PairTable<M, PIN, PO>;
    PT t{};
    constexpr const auto& b = BasisHolder<M, PO>::b;
    int q = 0;
    for (int j = 0; j < PT::P; ++j) {
        t.jptr[j] = q;
        for (int ii = 0; ii < PT::LI; ++ii)
            for (int k = 0; k < PT::P; ++k) {
                long long m0 = triple<M, PIN, PO>(b, ii, j, k);
                long long m1 = (PT::LI + ii < PT::L) ? triple<M, PIN, PO>(b, PT::LI + ii, j, k) : 0;
                if (m0 != 0 || m1 != 0) {
                    t.ii[q] = ii; t.k[q] = k; t.m0[q] = (double)m0; t.m1[q] = (double)m1;
                    ++q;
                }
            }
    }
    t.jptr[PT::P] = q;
    return t;
}

template <int M, int PIN, int PO>
struct PairHolder {
    static constexpr PairTable<M, PIN, PO> t = make_pair_table<M, PIN, PO>();
};

}  // namespace tab
}  // namespace sg
