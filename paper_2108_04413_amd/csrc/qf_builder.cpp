// Host-side builder of the Jordan-Wigner Pauli tables (qf_build_paulis).
//
// Route: every ladder operator is written in the "ordered" form
// X^x Z^z (X factors to the left of Z factors), in which the JW images of
// Sec. 2.2, Eqs. (13)-(14) have real coefficients:
//     a_p         = 1/2 X_p (1 - Z_p) Z_{p-1}..Z_0
//     a_p^dagger  = 1/2 X_p (1 + Z_p) Z_{p-1}..Z_0
// Products of ordered strings only pick up signs,
//     (X^a Z^b)(X^c Z^d) = (-1)^popcount(b & c) X^(a^c) Z^(b^d),
// so a whole operator is a real-weighted sum of ordered strings.  At the end
// X^x Z^z = i^-popcount(x & z) P(x, z) converts to Hermitian Pauli strings.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>
#include <vector>

#include "qf_common.h"

namespace qf {

std::string &last_error()
{
    static thread_local std::string msg;
    return msg;
}

namespace {

struct Key {
    uint64_t x, z;
    bool operator==(const Key &o) const { return x == o.x && z == o.z; }
    bool operator<(const Key &o) const { return x != o.x ? x < o.x : z < o.z; }
};

struct KeyHash {
    size_t operator()(const Key &k) const
    {
        uint64_t h = k.x * 0x9E3779B97F4A7C15ull ^ (k.z + 0x632BE59BD9B4E019ull + (k.x << 6));
        return (size_t)(h ^ (h >> 29));
    }
};

using Accum = std::unordered_map<Key, double, KeyHash>;

struct Ladder {
    int p;
    bool dagger;
};

// Add w * (product of ladder ops, leftmost first) into acc, ordered form.
void expand_product(const Ladder *ops, int m, double w, Accum &acc)
{
    const int nterm = 1 << m;
    for (int choice = 0; choice < nterm; choice++) {
        uint64_t x = 0, z = 0;
        double v = w;
        for (int j = 0; j < m; j++) {
            const uint64_t bit = 1ull << ops[j].p;
            const uint64_t chain = bit - 1;
            const bool with_z = (choice >> j) & 1;
            // factor: X^bit Z^(chain | [bit]) with weight 1/2 or +-1/2
            const uint64_t fx = bit, fz = with_z ? (chain | bit) : chain;
            double fw = 0.5;
            if (with_z && !ops[j].dagger)
                fw = -0.5;
            if (popc64(z & fx) & 1)
                v = -v;
            x ^= fx;
            z ^= fz;
            v *= fw;
        }
        acc[Key{x, z}] += v;
    }
}

// Phase exponent of X^x Z^z in terms of P(x, z): X^x Z^z = i^-a P(x,z), a = popcount(x & z).
inline int ordered_phase(uint64_t x, uint64_t z) { return popc64(x & z) & 3; }

struct Built {
    std::vector<qf_term> terms;
    std::vector<int64_t> off;
    std::vector<int64_t> kept;
};

void build_hamiltonian(int n, const double *h, const double *g, double e_core, Built &out)
{
    const int N = 2 * n;
    Accum acc;
    acc.reserve(1 << 16);
    if (e_core != 0.0)
        acc[Key{0, 0}] += e_core;
    // one-body: h_PQ a+_P a_Q, spins equal
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++) {
            const double v = h[p * n + q];
            if (v == 0.0)
                continue;
            for (int s = 0; s < 2; s++) {
                Ladder ops[2] = {{2 * p + s, true}, {2 * q + s, false}};
                expand_product(ops, 2, v, acc);
            }
        }
    // two-body, physicists' form: 1/2 sum <PQ|RS> a+_P a+_Q a_S a_R with
    // <PQ|RS> = (pr|qs) for spin(P) = spin(R), spin(Q) = spin(S).  This equals
    // the antisymmetrized 1/4 sum <PQ||RS> form of Eq. (1).
    for (int p = 0; p < n; p++)
        for (int r = 0; r < n; r++)
            for (int q = 0; q < n; q++)
                for (int s = 0; s < n; s++) {
                    const double v = g[((size_t)(p * n + r) * n + q) * n + s];
                    if (v == 0.0)
                        continue;
                    for (int sa = 0; sa < 2; sa++)
                        for (int sb = 0; sb < 2; sb++) {
                            const int P = 2 * p + sa, R = 2 * r + sa, Q = 2 * q + sb, S = 2 * s + sb;
                            if (P == Q || R == S)
                                continue;
                            Ladder ops[4] = {{P, true}, {Q, true}, {S, false}, {R, false}};
                            expand_product(ops, 4, 0.5 * v, acc);
                        }
                }
    std::vector<std::pair<Key, double>> items(acc.begin(), acc.end());
    std::sort(items.begin(), items.end(),
              [](const std::pair<Key, double> &a, const std::pair<Key, double> &b) { return a.first < b.first; });
    (void)N;
    for (auto &it : items) {
        const int a = ordered_phase(it.first.x, it.first.z);
        // coefficient of P(x,z) = w * i^-a
        if (a & 1) {
            if (std::fabs(it.second) > 1e-12)
                raise(QF_E_NOTHERM, "Hamiltonian string with imaginary coefficient");
            continue;
        }
        const double c = (a == 2) ? -it.second : it.second;
        if (std::fabs(c) <= 1e-12)
            continue;
        out.terms.push_back(qf_term{it.first.x, it.first.z, c});
    }
    out.off.push_back(0);
    for (size_t i = 1; i < out.terms.size(); i++)
        if (out.terms[i].x != out.terms[i - 1].x)
            out.off.push_back((int64_t)i);
    out.off.push_back((int64_t)out.terms.size());
}

struct Excitation {
    uint64_t det;
    int ncre;
    int cre[2];  // a, b
    int ann[2];  // j, i  (tau = a+_a a+_b a_j a_i)
};

std::vector<Excitation> enumerate(int nq, int ne, bool singles, bool doubles)
{
    std::vector<Excitation> ex;
    const uint64_t ref = ne >= 64 ? ~0ull : ((1ull << ne) - 1);
    if (singles)
        for (int i = 0; i < ne; i++)
            for (int a = ne; a < nq; a++)
                if ((i & 1) == (a & 1))
                    ex.push_back({ref ^ (1ull << i) ^ (1ull << a), 1, {a, -1}, {i, -1}});
    if (doubles)
        for (int i = 0; i < ne; i++)
            for (int j = i + 1; j < ne; j++)
                for (int a = ne; a < nq; a++)
                    for (int b = a + 1; b < nq; b++)
                        if ((i & 1) + (j & 1) == (a & 1) + (b & 1))
                            ex.push_back({ref ^ (1ull << i) ^ (1ull << j) ^ (1ull << a) ^ (1ull << b), 2,
                                          {a, b}, {j, i}});
    std::stable_sort(ex.begin(), ex.end(),
                     [](const Excitation &u, const Excitation &v) { return u.det < v.det; });
    return ex;
}

// Emit the strings of JW(kappa) = i sum c_k P_k for kappa = tau - tau^dagger.
void emit_kappa(const Excitation &e, std::vector<qf_term> &out)
{
    Accum acc;
    const int m = 2 * e.ncre;
    Ladder tau[4], dag[4];
    int t = 0;
    for (int c = 0; c < e.ncre; c++)
        tau[t++] = {e.cre[c], true};
    for (int c = 0; c < e.ncre; c++)
        tau[t++] = {e.ann[c], false};
    // tau^dagger: reverse order, daggers flipped
    for (int j = 0; j < m; j++)
        dag[j] = {tau[m - 1 - j].p, !tau[m - 1 - j].dagger};
    expand_product(tau, m, 1.0, acc);
    expand_product(dag, m, -1.0, acc);
    std::vector<std::pair<Key, double>> items(acc.begin(), acc.end());
    std::sort(items.begin(), items.end(),
              [](const std::pair<Key, double> &a, const std::pair<Key, double> &b) { return a.first < b.first; });
    for (auto &it : items) {
        const int a = ordered_phase(it.first.x, it.first.z);
        // coefficient of P = w i^-a must equal i c  ->  c = w i^(-a-1)
        if (!(a & 1)) {
            if (std::fabs(it.second) > 1e-12)
                raise(QF_E_NOTHERM, "kappa string with a real coefficient");
            continue;
        }
        const double c = (a == 1) ? -it.second : it.second;
        if (std::fabs(c) <= 1e-12)
            continue;
        out.push_back(qf_term{it.first.x, it.first.z, c});
    }
}

// Generalized singles and doubles of an ADAPT pool (Sec. 3.2): every
// S_z-conserving tau = a+_p a_q (p > q) and tau = a+_p a+_q a_s a_r with
// p < q, r < s and (p, q) after (r, s), regardless of occupation; singles
// first, ordered by (q, p), then doubles by ((r, s), (p, q)).
std::vector<Excitation> generalized_pool(int nq)
{
    std::vector<Excitation> ex;
    for (int q = 0; q < nq; q++)
        for (int p = q + 1; p < nq; p++)
            if (((p ^ q) & 1) == 0)
                ex.push_back({0, 1, {p, -1}, {q, -1}});
    for (int r = 0; r < nq; r++)
        for (int s = r + 1; s < nq; s++)
            for (int p = r; p < nq; p++)
                for (int q = p + 1; q < nq; q++) {
                    if (p == r && q <= s)
                        continue;
                    if ((p & 1) + (q & 1) != (r & 1) + (s & 1))
                        continue;
                    ex.push_back({0, 2, {p, q}, {s, r}});
                }
    return ex;
}

void build_ansatz(int kind, int n_orb, int ne, const double *t_rank, int64_t top_k, Built &out)
{
    const int nq = 2 * n_orb;
    std::vector<Excitation> ex;
    std::vector<int64_t> idx;
    if (kind == QF_GSD_POOL) {
        ex = generalized_pool(nq);
        for (size_t m = 0; m < ex.size(); m++)
            idx.push_back((int64_t)m);
    } else if (kind == QF_PUCCD) {
        const int nocc = ne / 2, nvir = (nq - ne) / 2;
        for (int i = 0; i < nocc; i++)
            for (int a = 0; a < nvir; a++) {
                const int ia = 2 * i, ib = 2 * i + 1, aa = 2 * nocc + 2 * a, ab = 2 * nocc + 2 * a + 1;
                // tau = a+_{a beta} a+_{a alpha} a_{i alpha} a_{i beta}
                Excitation e{0, 2, {ab, aa}, {ia, ib}};
                ex.push_back(e);
                idx.push_back((int64_t)idx.size());
            }
    } else {
        ex = enumerate(nq, ne, kind == QF_UCCSD, true);
        for (size_t m = 0; m < ex.size(); m++)
            idx.push_back((int64_t)m);
        if (kind == QF_UCCD_TOP) {
            std::vector<int64_t> order(ex.size());
            for (size_t m = 0; m < ex.size(); m++)
                order[m] = (int64_t)m;
            std::stable_sort(order.begin(), order.end(), [&](int64_t u, int64_t v) {
                return std::fabs(t_rank[u]) > std::fabs(t_rank[v]);
            });
            if ((size_t)top_k < order.size())
                order.resize((size_t)top_k);
            std::sort(order.begin(), order.end());
            std::vector<Excitation> keep;
            for (int64_t m : order)
                keep.push_back(ex[(size_t)m]);
            ex.swap(keep);
            idx = order;
        }
    }
    out.off.push_back(0);
    for (auto &e : ex) {
        emit_kappa(e, out.terms);
        out.off.push_back((int64_t)out.terms.size());
    }
    out.kept = idx;
}

// The excitations of an ansatz kind, in emission order (as build_ansatz).
std::vector<Excitation> ansatz_excitations(int kind, int n_orb, int ne, const double *t_rank, int64_t top_k)
{
    const int nq = 2 * n_orb;
    if (kind == QF_GSD_POOL)
        return generalized_pool(nq);
    if (kind == QF_PUCCD) {
        std::vector<Excitation> ex;
        const int nocc = ne / 2, nvir = (nq - ne) / 2;
        for (int i = 0; i < nocc; i++)
            for (int a = 0; a < nvir; a++) {
                const int ia = 2 * i, ib = 2 * i + 1, aa = 2 * nocc + 2 * a, ab = 2 * nocc + 2 * a + 1;
                ex.push_back(Excitation{0, 2, {ab, aa}, {ia, ib}});
            }
        return ex;
    }
    std::vector<Excitation> ex = enumerate(nq, ne, kind == QF_UCCSD, true);
    if (kind == QF_UCCD_TOP) {
        std::vector<int64_t> order(ex.size());
        for (size_t m = 0; m < ex.size(); m++)
            order[m] = (int64_t)m;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t u, int64_t v) { return std::fabs(t_rank[u]) > std::fabs(t_rank[v]); });
        if ((size_t)top_k < order.size())
            order.resize((size_t)top_k);
        std::sort(order.begin(), order.end());
        std::vector<Excitation> keep;
        for (int64_t m : order)
            keep.push_back(ex[(size_t)m]);
        ex.swap(keep);
    }
    return ex;
}

// tau |ref> = sign |det>: the ladder operators act right to left, a_p and
// a+_p each contribute (-1)^(occupied spin orbitals below p); sign 0 if tau
// annihilates the reference.
void excite(uint64_t ref, const Excitation &e, uint64_t &det, int &sign)
{
    int ops[4];
    bool cre[4];
    int m = 0;
    for (int c = 0; c < e.ncre; c++) {
        ops[m] = e.cre[c];
        cre[m++] = true;
    }
    for (int c = 0; c < e.ncre; c++) {
        ops[m] = e.ann[c];
        cre[m++] = false;
    }
    uint64_t b = ref;
    int s = 1;
    for (int j = m - 1; j >= 0; j--) {
        const uint64_t bit = 1ull << ops[j];
        if (((b & bit) != 0) == cre[j]) {
            det = 0;
            sign = 0;
            return;
        }
        if (popc64(b & (bit - 1)) & 1)
            s = -s;
        b ^= bit;
    }
    det = b;
    sign = s;
}

} // namespace
} // namespace qf

using namespace qf;

extern "C" int qf_excited_determinants(int kind, int n_orb, int n_elec, const double *t_rank, int64_t top_k,
                                       uint64_t *det, int *sign, int64_t cap, int64_t *n_out)
{
    return guarded([&]() -> int {
        if (kind < QF_UCCSD || kind > QF_GSD_POOL)
            return fail(QF_E_ARG, "qf_excited_determinants: not an ansatz kind: %d", kind);
        if (n_orb < 1 || 2 * n_orb > 64 || n_elec < 0 || n_elec > 2 * n_orb)
            return fail(QF_E_RANGE, "qf_excited_determinants: n_orb=%d n_elec=%d out of range", n_orb, n_elec);
        if (!n_out || (kind == QF_UCCD_TOP && (!t_rank || top_k < 0)))
            return fail(QF_E_ARG, "qf_excited_determinants: bad arguments");
        const std::vector<Excitation> ex = ansatz_excitations(kind, n_orb, n_elec, t_rank, top_k);
        *n_out = (int64_t)ex.size();
        if (!det)
            return QF_OK;
        if (!sign || cap < *n_out)
            return fail(QF_E_SIZE, "qf_excited_determinants: need %lld entries", (long long)*n_out);
        const uint64_t ref = n_elec >= 64 ? ~0ull : ((1ull << n_elec) - 1);
        for (size_t m = 0; m < ex.size(); m++)
            excite(ref, ex[m], det[m], sign[m]);
        return QF_OK;
    });
}

extern "C" int qf_excitations(int kind, int n_orb, int n_elec, const double *t_rank, int64_t top_k, int32_t *ops,
                              int64_t cap, int64_t *n_out)
{
    return guarded([&]() -> int {
        if (kind < QF_UCCSD || kind > QF_GSD_POOL)
            return fail(QF_E_ARG, "qf_excitations: not an ansatz kind: %d", kind);
        if (n_orb < 1 || 2 * n_orb > 64 || n_elec < 0 || n_elec > 2 * n_orb)
            return fail(QF_E_RANGE, "qf_excitations: n_orb=%d n_elec=%d out of range", n_orb, n_elec);
        if (!n_out || (kind == QF_UCCD_TOP && (!t_rank || top_k < 0)))
            return fail(QF_E_ARG, "qf_excitations: bad arguments");
        const std::vector<Excitation> ex = ansatz_excitations(kind, n_orb, n_elec, t_rank, top_k);
        *n_out = (int64_t)ex.size();
        if (!ops)
            return QF_OK;
        if (cap < *n_out)
            return fail(QF_E_SIZE, "qf_excitations: need %lld entries", (long long)*n_out);
        for (size_t m = 0; m < ex.size(); m++) {
            int32_t *o = ops + 4 * m;
            o[0] = ex[m].cre[0];
            o[1] = ex[m].ncre > 1 ? ex[m].cre[1] : -1;
            o[2] = ex[m].ann[0];
            o[3] = ex[m].ncre > 1 ? ex[m].ann[1] : -1;
        }
        return QF_OK;
    });
}

extern "C" int qf_mp_denominators(int kind, int n_orb, int n_elec, const double *h, const double *g,
                                  const double *t_rank, int64_t top_k, double *delta, int64_t cap, int64_t *n_out)
{
    return guarded([&]() -> int {
        if (kind < QF_UCCSD || kind > QF_PUCCD)
            return fail(QF_E_ARG, "qf_mp_denominators: not a particle-hole ansatz kind: %d", kind);
        if (n_orb < 1 || 2 * n_orb > 64 || n_elec < 0 || n_elec > 2 * n_orb)
            return fail(QF_E_RANGE, "qf_mp_denominators: n_orb=%d n_elec=%d out of range", n_orb, n_elec);
        if (!n_out || !h || !g || (kind == QF_UCCD_TOP && (!t_rank || top_k < 0)))
            return fail(QF_E_ARG, "qf_mp_denominators: bad arguments");
        const std::vector<Excitation> ex = ansatz_excitations(kind, n_orb, n_elec, t_rank, top_k);
        *n_out = (int64_t)ex.size();
        if (!delta)
            return QF_OK;
        if (cap < *n_out)
            return fail(QF_E_SIZE, "qf_mp_denominators: need %lld entries", (long long)*n_out);
        // reference Fock diagonal: eps_P = h_pp + sum_{J occ} [(pp|jj) - d(sP,sJ) (pj|jp)]
        const int n = n_orb, N = 2 * n_orb;
        std::vector<double> eps((size_t)N);
        for (int P = 0; P < N; P++) {
            const int p = P / 2;
            double e = h[p * n + p];
            for (int J = 0; J < n_elec; J++) {
                const int j = J / 2;
                e += g[((size_t)(p * n + p) * n + j) * n + j];
                if ((P & 1) == (J & 1))
                    e -= g[((size_t)(p * n + j) * n + j) * n + p];
            }
            eps[(size_t)P] = e;
        }
        for (size_t m = 0; m < ex.size(); m++) {
            double d = 0.0;
            for (int c = 0; c < ex[m].ncre; c++)
                d += eps[(size_t)ex[m].ann[c]] - eps[(size_t)ex[m].cre[c]];
            delta[m] = d;
        }
        return QF_OK;
    });
}

extern "C" int qf_build_paulis(int kind, int n_orb, int n_elec, const double *h, const double *g,
                               double e_core, const double *t_rank, int64_t top_k,
                               qf_term *out, int64_t cap, int64_t *n_out,
                               int64_t *off, int64_t off_cap, int64_t *n_off, int64_t *kept)
{
    return guarded([&]() -> int {
        if (kind < QF_HAMILTONIAN || kind > QF_GSD_POOL)
            return fail(QF_E_ARG, "qf_build_paulis: unknown kind %d", kind);
        if (n_orb < 1 || 2 * n_orb > 64)
            return fail(QF_E_RANGE, "qf_build_paulis: n_orb=%d out of range [1, 32]", n_orb);
        if (n_elec < 0 || n_elec > 2 * n_orb)
            return fail(QF_E_RANGE, "qf_build_paulis: n_elec=%d out of range", n_elec);
        if (!n_out || !n_off)
            return fail(QF_E_ARG, "qf_build_paulis: n_out and n_off must not be NULL");
        if (kind == QF_HAMILTONIAN && (!h || !g))
            return fail(QF_E_ARG, "qf_build_paulis: Hamiltonian needs h and g");
        if (kind == QF_UCCD_TOP && (!t_rank || top_k < 0))
            return fail(QF_E_ARG, "qf_build_paulis: QF_UCCD_TOP needs t_rank and top_k >= 0");
        if (out && (!off || cap < 0 || off_cap < 0))
            return fail(QF_E_ARG, "qf_build_paulis: bad output buffers");
        Built b;
        if (kind == QF_HAMILTONIAN)
            build_hamiltonian(n_orb, h, g, e_core, b);
        else
            build_ansatz(kind, n_orb, n_elec, t_rank, top_k, b);
        *n_out = (int64_t)b.terms.size();
        *n_off = (int64_t)b.off.size();
        if (!out)
            return QF_OK;
        if (cap < *n_out || off_cap < *n_off)
            return fail(QF_E_SIZE, "qf_build_paulis: need %lld terms and %lld offsets",
                        (long long)*n_out, (long long)*n_off);
        std::memcpy(out, b.terms.data(), b.terms.size() * sizeof(qf_term));
        std::memcpy(off, b.off.data(), b.off.size() * sizeof(int64_t));
        if (kept && kind != QF_HAMILTONIAN)
            std::memcpy(kept, b.kept.data(), b.kept.size() * sizeof(int64_t));
        return QF_OK;
    });
}

extern "C" int qf_ansatz_angles(const qf_term *A, const int64_t *exc_off, int64_t n_par,
                                const double *t, double *theta)
{
    if (n_par < 0 || (n_par > 0 && (!A || !exc_off || !t || !theta)))
        return fail(QF_E_ARG, "qf_ansatz_angles: bad arguments");
    for (int64_t mu = 0; mu < n_par; mu++)
        for (int64_t k = exc_off[mu]; k < exc_off[mu + 1]; k++)
            theta[k] = -A[k].c * t[mu];
    return QF_OK;
}

extern "C" int qf_grad_t(const qf_term *A, const int64_t *exc_off, int64_t n_par,
                         const double *dE_dtheta, double *dE_dt)
{
    if (n_par < 0 || (n_par > 0 && (!A || !exc_off || !dE_dtheta || !dE_dt)))
        return fail(QF_E_ARG, "qf_grad_t: bad arguments");
    for (int64_t mu = 0; mu < n_par; mu++) {
        double s = 0.0;
        for (int64_t k = exc_off[mu]; k < exc_off[mu + 1]; k++)
            s += -A[k].c * dE_dtheta[k];
        dE_dt[mu] = s;
    }
    return QF_OK;
}

extern "C" const char *qf_last_error(void) { return qf::last_error().c_str(); }

extern "C" const char *qf_version(void) { return "qforte-mi355x 0.10 (gfx950)"; }
