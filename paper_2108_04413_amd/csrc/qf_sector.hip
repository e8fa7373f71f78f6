// Particle-number and S_z restricted state vector (the restriction the
// paper's conclusion names for going past ~24 qubits), on gfx950.
//
// Only determinants with N_alpha alpha and N_beta beta electrons are stored:
// an alpha (beta) string is the n_orb-bit mask of the occupied alpha (beta)
// orbitals (spin orbital 2j = alpha, 2j + 1 = beta of spatial orbital j);
// strings of one spin are ranked in increasing order and determinant (a, b)
// lives at rank(a) * D_beta + rank(b).  Each spin keeps its string list and
// a rank table indexed by the whole n_orb-bit mask (~0u: wrong occupation),
// so a flip of occupied orbitals is mapped back to an index by two lookups.
//
// Work is tiled by rows: a tile is one alpha string and 256 consecutive beta
// strings, so every test on the alpha part (is the row inside an
// excitation's domain, is the flipped row inside the sector) is uniform
// across the workgroup and rows outside are skipped without memory access.
//   k_sector_prepare  psi = |reference>.
//   k_sector_rotate   one factor exp(t kappa) of Sec. 3.1: each determinant
//                     D with tau D = s D' (s the fermionic sign) is rotated
//                     with D' (D -> cos t D + s sin t D').
//   k_sector_energy   <psi|H|psi> over the grouped Pauli strings: for every
//                     stored y and group g with y ^ x_g stored,
//                     conj(psi[y ^ x_g]) D_g(y) psi[y] (Eq. (17)); each
//                     thread holds its amplitude and walks all groups.
//   k_sector_sigma    lambda = H psi in the sector: lambda[y] = sum_g
//                     D_g(y ^ x_g) psi[y ^ x_g] over stored partners, fused
//                     with E = Re <psi|lambda>.
//   k_sector_adjoint  one step of the reverse sweep for one dUCC factor:
//                     dE/dt_mu = 2 Re <lambda|kappa_mu|phi> over its
//                     determinant pairs, then phi and lambda rotated back by
//                     -t_mu (the factor undone).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "qf_common.h"
#include "qf_host.h"
#include "qf_kernels.h"

namespace qf {

constexpr int kSecT = 256;        // beta strings per tile (one workgroup)
constexpr uint32_t kNoRank = ~0u;

// One excitation tau = a+_{c0} a+_{c1} a_{a0} a_{a1} (unused slots -1):
// its masks split by spin, and the operators in the order they act.
struct SecExc {
    uint32_t annA, annB, creA, creB;  // compacted alpha / beta orbital masks
    int32_t op[4];                    // spin orbitals, right to left
    int32_t dag[4];                   // 1: creation
    int32_t nops;
    int32_t pad;
};

// A flip-mask group restricted to the sector: x and each string's z split by
// spin; coefficients with the phase i^popcount(x & z) folded in (real-phase
// strings [k0, kre), imaginary-phase [kre, k1)).
struct SecGroup {
    uint32_t xA, xB;
    int32_t k0, kre, k1;
    uint32_t halfA;  // popcount(xA) / 2: a row maps into the sector iff popcount(a & xA) == halfA
};

struct SecStr {
    uint32_t zA, zB;
    double c;
};

// (-1)^(occupied spin orbitals below spin orbital p) for the determinant
// (a, b): alpha orbitals j' < j, beta orbitals j' < j, and for a beta spin
// orbital also the alpha of its own spatial orbital.
__device__ __forceinline__ uint32_t below_parity(uint32_t a, uint32_t b, int p)
{
    const int j = p >> 1;
    const uint32_t lo = (1u << j) - 1u;
    uint32_t c = __popc(a & lo) + __popc(b & lo);
    if (p & 1)
        c += (a >> j) & 1u;
    return c & 1u;
}

__global__ __launch_bounds__(kBlock) void k_sector_prepare(double2 *__restrict__ psi, uint64_t dim, uint64_t at)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += stride)
        psi[i] = make_double2(i == at ? 1.0 : 0.0, 0.0);
}

__global__ __launch_bounds__(kSecT) void k_sector_rotate(double2 *__restrict__ psi, const uint32_t *__restrict__ strA,
                                                         const uint32_t *__restrict__ strB,
                                                         const uint32_t *__restrict__ rankA,
                                                         const uint32_t *__restrict__ rankB, const uint32_t *__restrict__ rows,
                                                         uint32_t nrows, uint32_t DB, SecExc e, double cs, double sn)
{
    const uint32_t nchunk = (DB + kSecT - 1) / kSecT;
    const uint64_t ntiles = (uint64_t)nrows * nchunk;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // the alpha strings of the domain of tau (host list)
        const uint32_t ia = rows[(uint32_t)(t / nchunk)], ch = (uint32_t)(t % nchunk);
        const uint32_t a = strA[ia];
        const uint32_t a2 = a ^ e.annA ^ e.creA;
        const uint32_t ia2 = rankA[a2];
        const uint32_t ib = ch * kSecT + threadIdx.x;
        if (ib >= DB)
            continue;
        const uint32_t b = strB[ib];
        if ((b & e.annB) != e.annB || (b & e.creB) != 0u)
            continue;
        const uint32_t b2 = b ^ e.annB ^ e.creB;
        const uint32_t ib2 = rankB[b2];
        // sign of tau |a, b>: the operators act right to left on the bit string
        uint32_t ca = a, cb = b, par = 0u;
        for (int k = 0; k < e.nops; k++) {
            const int p = e.op[k];
            par ^= below_parity(ca, cb, p);
            if (p & 1)
                cb ^= 1u << (p >> 1);
            else
                ca ^= 1u << (p >> 1);
        }
        const double s = par ? -sn : sn;
        const uint64_t i1 = (uint64_t)ia * DB + ib, i2 = (uint64_t)ia2 * DB + ib2;
        const double2 u = psi[i1], v = psi[i2];
        psi[i1] = make_double2(cs * u.x - s * v.x, cs * u.y - s * v.y);
        psi[i2] = make_double2(cs * v.x + s * u.x, cs * v.y + s * u.y);
    }
}

__global__ __launch_bounds__(kSecT) void k_sector_energy(const double2 *__restrict__ psi,
                                                         const uint32_t *__restrict__ strA,
                                                         const uint32_t *__restrict__ strB,
                                                         const uint32_t *__restrict__ rankA,
                                                         const uint32_t *__restrict__ rankB, uint32_t DA,
                                                         uint32_t DB, const SecGroup *__restrict__ groups, int G,
                                                         const SecStr *__restrict__ strs, double *partials,
                                                         unsigned *counter, double *out)
{
    double acc[1] = {0.0};
    const uint32_t nchunk = (DB + kSecT - 1) / kSecT;
    const uint64_t ntiles = (uint64_t)DA * nchunk;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t ia = (uint32_t)(t / nchunk), ch = (uint32_t)(t % nchunk);
        const uint32_t a = strA[ia];
        const uint32_t ib = ch * kSecT + threadIdx.x;
        const bool live = ib < DB;
        const uint32_t b = live ? strB[ib] : 0u;
        const double2 v = live ? psi[(uint64_t)ia * DB + ib] : make_double2(0.0, 0.0);
        for (int g = 0; g < G; g++) {
            const SecGroup gd = groups[g];
            // uniform: does the alpha flip keep this row in the sector?
            if ((uint32_t)__popc(a & gd.xA) != gd.halfA)
                continue;
            const uint32_t ia2 = gd.xA ? rankA[a ^ gd.xA] : ia;
            const uint32_t ib2 = gd.xB ? (live ? rankB[b ^ gd.xB] : kNoRank) : ib;
            if (!live || ib2 == kNoRank)
                continue;
            double dr = 0.0, di = 0.0;
            for (int k = gd.k0; k < gd.kre; k++) {
                const SecStr z = strs[k];
                dr += ((__popc(a & z.zA) + __popc(b & z.zB)) & 1u) ? -z.c : z.c;
            }
            for (int k = gd.kre; k < gd.k1; k++) {
                const SecStr z = strs[k];
                di += ((__popc(a & z.zA) + __popc(b & z.zB)) & 1u) ? -z.c : z.c;
            }
            const double2 w = psi[(uint64_t)ia2 * DB + ib2];
            // Re(conj(w) (dr + i di) v)
            acc[0] += dr * (w.x * v.x + w.y * v.y) - di * (w.x * v.y - w.y * v.x);
        }
    }
    // block sum, then the last block sums the partials in block order
    __shared__ double lds[kSecT / 64];
    __shared__ bool last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s = acc[0];
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off, 64);
    if (lane == 0)
        lds[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bsum = 0.0;
        for (int w = 0; w < kSecT / 64; w++)
            bsum += lds[w];
        __hip_atomic_store(&partials[blockIdx.x], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    __shared__ double red[kSecT];
    double p = 0.0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += kSecT)
        p += __hip_atomic_load(&partials[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    red[threadIdx.x] = p;
    __syncthreads();
    for (int w = kSecT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0];
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Fixed-order block sum of one value, then the last block to arrive sums the
// per-block partials in block order into *out.
__device__ __forceinline__ void sector_reduce(double v, double *partials, unsigned *counter, double *out)
{
    __shared__ double lds[kSecT / 64];
    __shared__ bool last;
    __shared__ double red[kSecT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bsum = 0.0;
        for (int w = 0; w < kSecT / 64; w++)
            bsum += lds[w];
        __hip_atomic_store(&partials[blockIdx.x], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    double p = 0.0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += kSecT)
        p += __hip_atomic_load(&partials[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    red[threadIdx.x] = p;
    __syncthreads();
    for (int w = kSecT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = red[0];
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Fixed-order block sum of one value into out (thread 0 stores it; no
// cross-workgroup step: k_sector_grad_reduce adds the workgroups later).
__device__ __forceinline__ void sector_block_sum(double v, double *out)
{
    __shared__ double lds[kSecT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bsum = 0.0;
        for (int w = 0; w < kSecT / 64; w++)
            bsum += lds[w];
        *out = bsum;
    }
}

__global__ __launch_bounds__(kSecT) void k_sector_sigma(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                                        const uint32_t *__restrict__ strA,
                                                        const uint32_t *__restrict__ strB,
                                                        const uint32_t *__restrict__ rankA,
                                                        const uint32_t *__restrict__ rankB, uint32_t DA,
                                                        uint32_t DB, const SecGroup *__restrict__ groups, int G,
                                                        const SecStr *__restrict__ strs, double *partials,
                                                        unsigned *counter, double *out)
{
    double acc = 0.0;
    const uint32_t nchunk = (DB + kSecT - 1) / kSecT;
    const uint64_t ntiles = (uint64_t)DA * nchunk;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t ia = (uint32_t)(t / nchunk), ch = (uint32_t)(t % nchunk);
        const uint32_t a = strA[ia];
        const uint32_t ib = ch * kSecT + threadIdx.x;
        const bool live = ib < DB;
        const uint32_t b = live ? strB[ib] : 0u;
        double lx = 0.0, ly = 0.0;
        for (int g = 0; g < G; g++) {
            const SecGroup gd = groups[g];
            if ((uint32_t)__popc(a & gd.xA) != gd.halfA)
                continue;
            const uint32_t a2 = a ^ gd.xA;
            const uint32_t ia2 = gd.xA ? rankA[a2] : ia;
            const uint32_t b2 = b ^ gd.xB;
            const uint32_t ib2 = gd.xB ? (live ? rankB[b2] : kNoRank) : ib;
            if (!live || ib2 == kNoRank)
                continue;
            // D_g at the partner determinant (a2, b2)
            double dr = 0.0, di = 0.0;
            for (int k = gd.k0; k < gd.kre; k++) {
                const SecStr z = strs[k];
                dr += ((__popc(a2 & z.zA) + __popc(b2 & z.zB)) & 1u) ? -z.c : z.c;
            }
            for (int k = gd.kre; k < gd.k1; k++) {
                const SecStr z = strs[k];
                di += ((__popc(a2 & z.zA) + __popc(b2 & z.zB)) & 1u) ? -z.c : z.c;
            }
            const double2 w = psi[(uint64_t)ia2 * DB + ib2];
            lx += dr * w.x - di * w.y;
            ly += dr * w.y + di * w.x;
        }
        if (live) {
            const uint64_t i = (uint64_t)ia * DB + ib;
            lam[i] = make_double2(lx, ly);
            const double2 v = psi[i];
            acc += v.x * lx + v.y * ly;
        }
    }
    sector_reduce(acc, partials, counter, out);
}

// grad_out = 2 Re <lam|kappa|phi> over the pairs (D, D' = tau D / s):
// kappa D = s D', kappa D' = -s D, so the pair adds
// s (conj(lam[D']) phi[D] - conj(lam[D]) phi[D']); then both states are
// rotated by -t on the pair (D -> cos t D - s sin t D' ...).
__global__ __launch_bounds__(kSecT) void k_sector_adjoint(double2 *__restrict__ phi, double2 *__restrict__ lam,
                                                          const uint32_t *__restrict__ strA,
                                                          const uint32_t *__restrict__ strB,
                                                          const uint32_t *__restrict__ rankA,
                                                          const uint32_t *__restrict__ rankB,
                                                          const uint32_t *__restrict__ rows, uint32_t nrows,
                                                          uint32_t DB, SecExc e, double cs, double sn,
                                                          double *part)
{
    double acc = 0.0;
    const uint32_t nchunk = (DB + kSecT - 1) / kSecT;
    const uint64_t ntiles = (uint64_t)nrows * nchunk;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t ia = rows[(uint32_t)(t / nchunk)], ch = (uint32_t)(t % nchunk);
        const uint32_t a = strA[ia];
        const uint32_t ia2 = rankA[a ^ e.annA ^ e.creA];
        const uint32_t ib = ch * kSecT + threadIdx.x;
        if (ib >= DB)
            continue;
        const uint32_t b = strB[ib];
        if ((b & e.annB) != e.annB || (b & e.creB) != 0u)
            continue;
        const uint32_t ib2 = rankB[b ^ e.annB ^ e.creB];
        uint32_t ca = a, cb = b, par = 0u;
        for (int k = 0; k < e.nops; k++) {
            const int p = e.op[k];
            par ^= below_parity(ca, cb, p);
            if (p & 1)
                cb ^= 1u << (p >> 1);
            else
                ca ^= 1u << (p >> 1);
        }
        const double sgn = par ? -1.0 : 1.0;
        const uint64_t i1 = (uint64_t)ia * DB + ib, i2 = (uint64_t)ia2 * DB + ib2;
        const double2 u = phi[i1], v = phi[i2], lu = lam[i1], lv = lam[i2];
        // s (Re conj(lv) u - Re conj(lu) v)
        acc += sgn * ((lv.x * u.x + lv.y * u.y) - (lu.x * v.x + lu.y * v.y));
        // undo: rotation by -t (sn is sin t)
        const double s = sgn * sn;
        phi[i1] = make_double2(cs * u.x + s * v.x, cs * u.y + s * v.y);
        phi[i2] = make_double2(cs * v.x - s * u.x, cs * v.y - s * u.y);
        lam[i1] = make_double2(cs * lu.x + s * lv.x, cs * lu.y + s * lv.y);
        lam[i2] = make_double2(cs * lv.x - s * lu.x, cs * lv.y - s * lu.y);
    }
    sector_block_sum(2.0 * acc, part + blockIdx.x);
}

// dE/dt of every excitation: the sum of its workgroups' partials
// part[part0[m] .. part0[m + 1]) in workgroup order
__global__ __launch_bounds__(kSecT) void k_sector_grad_reduce(const double *__restrict__ part,
                                                              const uint32_t *__restrict__ part0, int E,
                                                              double *__restrict__ grad)
{
    const int m = blockIdx.x * kSecT + threadIdx.x;
    if (m >= E)
        return;
    double v = 0.0;
    for (uint32_t b = part0[m]; b < part0[m + 1]; b++)
        v += part[b];
    grad[m] = v;
}

uint32_t compact(uint64_t so, int spin, int n_orb)
{
    uint32_t m = 0;
    for (int j = 0; j < n_orb; j++)
        m |= (uint32_t)((so >> (2 * j + spin)) & 1ull) << j;
    return m;
}

} // namespace qf

struct qf_sector {
    int n_orb = 0, na = 0, nb = 0;
    uint32_t DA = 0, DB = 0;
    std::vector<uint32_t> strA, strB, rankA, rankB;
    std::vector<qf::SecExc> exc;
    int G = 0;
    uint32_t *d_strA = nullptr, *d_strB = nullptr, *d_rankA = nullptr, *d_rankB = nullptr;
    qf::SecGroup *d_groups = nullptr;
    qf::SecStr *d_strs = nullptr;
    double *d_partials = nullptr, *d_result = nullptr;
    unsigned *d_counter = nullptr;
    double *d_grad = nullptr;  // dE/dt of the last gradient call
    size_t grad_cap = 0;
    // per excitation, the alpha strings of its domain (rows[row0[m] ..
    // row0[m + 1]), alpha-string indices): launches cover those rows only
    std::vector<uint32_t> row0;
    uint32_t *d_rows = nullptr;
    // per excitation, its adjoint workgroups' partial sums part[part0[m] ..]
    std::vector<uint32_t> part0;
    uint32_t *d_part0 = nullptr;
    double *d_part = nullptr;
    ~qf_sector()
    {
        void *bufs[] = {d_strA, d_strB, d_rankA, d_rankB, d_groups, d_strs, d_partials, d_result, d_counter, d_grad,
                        d_rows, d_part0, d_part};
        for (void *p : bufs)
            if (p)
                (void)hipFree(p);
    }
};

namespace qf {
namespace {

constexpr int kSecGrid = 2048;

void strings_of(int n_orb, int k, std::vector<uint32_t> &str, std::vector<uint32_t> &rank)
{
    rank.assign((size_t)1 << n_orb, kNoRank);
    str.clear();
    for (uint32_t m = 0; m < (1u << n_orb); m++)
        if (__builtin_popcount(m) == k) {
            rank[m] = (uint32_t)str.size();
            str.push_back(m);
        }
}

template <class T> T *upload_new(const std::vector<T> &v)
{
    T *p = dev_alloc<T>(std::max<size_t>(v.size(), 1));
    if (!v.empty())
        QF_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

void sector_init(qf_sector &S, int n_orb, int na, int nb, const int32_t *exc, int64_t n_exc, const qf_term *H,
                 const int64_t *goff, int64_t G)
{
    if (n_orb < 1 || n_orb > 20)
        raise(QF_E_RANGE, "sector: n_orb=" + std::to_string(n_orb) + " out of range [1, 20]");
    if (na < 0 || na > n_orb || nb < 0 || nb > n_orb)
        raise(QF_E_RANGE, "sector: electron counts out of range");
    if (n_exc < 0 || G < 0 || (n_exc > 0 && !exc) || (G > 0 && (!H || !goff)))
        raise(QF_E_ARG, "sector: bad excitation or Hamiltonian arrays");
    S.n_orb = n_orb;
    S.na = na;
    S.nb = nb;
    strings_of(n_orb, na, S.strA, S.rankA);
    strings_of(n_orb, nb, S.strB, S.rankB);
    S.DA = (uint32_t)S.strA.size();
    S.DB = (uint32_t)S.strB.size();
    const int N = 2 * n_orb;
    for (int64_t m = 0; m < n_exc; m++) {
        const int32_t *o = exc + 4 * m;
        SecExc e;
        std::memset(&e, 0, sizeof e);
        // tau = a+_{o0} a+_{o1} a_{o2} a_{o3}: acting right to left
        const int order[4] = {3, 2, 1, 0};
        uint64_t cre = 0, ann = 0;
        for (int q : order) {
            const int p = o[q];
            if (p < 0)
                continue;
            if (p >= N)
                raise(QF_E_RANGE, "sector: excitation " + std::to_string(m) + " has a spin orbital >= 2 n_orb");
            const bool dag = q < 2;
            const uint64_t bit = 1ull << p;
            if ((dag ? cre : ann) & bit)
                raise(QF_E_ARG, "sector: excitation " + std::to_string(m) + " repeats an operator");
            (dag ? cre : ann) |= bit;
            e.op[e.nops] = p;
            e.dag[e.nops] = dag ? 1 : 0;
            e.nops++;
        }
        if (cre & ann)
            raise(QF_E_ARG, "sector: excitation " + std::to_string(m) + " creates and annihilates one orbital");
        e.creA = compact(cre, 0, n_orb);
        e.creB = compact(cre, 1, n_orb);
        e.annA = compact(ann, 0, n_orb);
        e.annB = compact(ann, 1, n_orb);
        if (__builtin_popcount(e.creA) != __builtin_popcount(e.annA) ||
            __builtin_popcount(e.creB) != __builtin_popcount(e.annB))
            raise(QF_E_ARG, "sector: excitation " + std::to_string(m) + " changes N_alpha or N_beta");
        S.exc.push_back(e);
    }
    if (G > 0) {
        std::vector<SecGroup> gd;
        std::vector<SecStr> st;
        for (int64_t g = 0; g < G; g++) {
            const uint64_t x = H[goff[g]].x;
            SecGroup d;
            std::memset(&d, 0, sizeof d);
            d.xA = compact(x, 0, n_orb);
            d.xB = compact(x, 1, n_orb);
            if (x >> N)
                raise(QF_E_RANGE, "sector: Hamiltonian mask has a bit >= 2 n_orb");
            // a flip of an odd number of one spin's orbitals never stays in the sector
            if ((__builtin_popcount(d.xA) & 1) || (__builtin_popcount(d.xB) & 1))
                continue;
            d.halfA = (uint32_t)__builtin_popcount(d.xA) / 2;
            std::vector<SecStr> re, im;
            for (int64_t k = goff[g]; k < goff[g + 1]; k++) {
                if (H[k].x != x)
                    raise(QF_E_ARG, "sector: group " + std::to_string(g) + " mixes flip masks");
                if (H[k].z >> N)
                    raise(QF_E_RANGE, "sector: Hamiltonian mask has a bit >= 2 n_orb");
                const int ph = __builtin_popcountll(x & H[k].z) & 3;
                SecStr s{compact(H[k].z, 0, n_orb), compact(H[k].z, 1, n_orb), (ph >= 2) ? -H[k].c : H[k].c};
                (ph & 1 ? im : re).push_back(s);
            }
            d.k0 = (int32_t)st.size();
            st.insert(st.end(), re.begin(), re.end());
            d.kre = (int32_t)st.size();
            st.insert(st.end(), im.begin(), im.end());
            d.k1 = (int32_t)st.size();
            gd.push_back(d);
        }
        S.G = (int)gd.size();
        S.d_groups = upload_new(gd);
        S.d_strs = upload_new(st);
    }
    std::vector<uint32_t> rows;
    S.row0.assign(1, 0u);
    for (const SecExc &e : S.exc) {
        for (uint32_t ia = 0; ia < S.DA; ia++) {
            const uint32_t a = S.strA[ia];
            if ((a & e.annA) == e.annA && (a & e.creA) == 0u)
                rows.push_back(ia);
        }
        if (rows.size() > (size_t)UINT32_MAX)
            raise(QF_E_SIZE, "sector: excitation domains too large");
        S.row0.push_back((uint32_t)rows.size());
    }
    S.d_rows = upload_new(rows);
    S.part0.assign(1, 0u);
    const uint32_t nchunk = (S.DB + kSecT - 1) / kSecT;
    for (size_t m = 0; m < S.exc.size(); m++) {
        const uint64_t tiles = (uint64_t)(S.row0[m + 1] - S.row0[m]) * nchunk;
        S.part0.push_back(S.part0.back() + (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, kSecGrid)));
    }
    S.d_part0 = upload_new(S.part0);
    S.d_part = dev_alloc<double>(std::max<size_t>(S.part0.back(), 1));
    S.d_strA = upload_new(S.strA);
    S.d_strB = upload_new(S.strB);
    S.d_rankA = upload_new(S.rankA);
    S.d_rankB = upload_new(S.rankB);
    S.d_partials = dev_alloc<double>(kSecGrid);
    S.d_result = dev_alloc<double>(1);
    S.d_counter = dev_alloc<unsigned>(1);
    QF_HIP(hipMemset(S.d_counter, 0, sizeof(unsigned)));
}

unsigned tile_grid(const qf_sector &S)
{
    const uint64_t tiles = (uint64_t)S.DA * ((S.DB + kSecT - 1) / kSecT);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(tiles, kSecGrid));
}

// workgroups for excitation m's domain rows
unsigned exc_grid(const qf_sector &S, size_t m)
{
    const uint64_t tiles = (uint64_t)(S.row0[m + 1] - S.row0[m]) * ((S.DB + kSecT - 1) / kSecT);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(tiles, kSecGrid));
}

} // namespace
} // namespace qf

using namespace qf;

extern "C" int qf_sector_create(int n_orb, int n_alpha, int n_beta, const int32_t *exc, int64_t n_exc,
                                const qf_term *H, const int64_t *group_off, int64_t n_groups, qf_sector **out)
{
    return guarded([&]() -> int {
        if (!out)
            return fail(QF_E_ARG, "qf_sector_create: out is NULL");
        *out = nullptr;
        qf_sector *S = new qf_sector();
        try {
            sector_init(*S, n_orb, n_alpha, n_beta, exc, n_exc, H, group_off, n_groups);
        } catch (...) {
            delete S;
            throw;
        }
        *out = S;
        return QF_OK;
    });
}

extern "C" int qf_sector_destroy(qf_sector *s)
{
    delete s;
    return QF_OK;
}

extern "C" int qf_sector_info(const qf_sector *s, int64_t *dim, int64_t *d_alpha, int64_t *d_beta,
                              int64_t *groups)
{
    if (!s)
        return fail(QF_E_ARG, "qf_sector_info: sector is NULL");
    if (dim)
        *dim = (int64_t)s->DA * (int64_t)s->DB;
    if (d_alpha)
        *d_alpha = s->DA;
    if (d_beta)
        *d_beta = s->DB;
    if (groups)
        *groups = s->G;
    return QF_OK;
}

extern "C" int qf_sector_prepare(qf_sector *s, void *psi, uint64_t occ_mask, void *stream)
{
    return guarded([&]() -> int {
        if (!s || !psi)
            return fail(QF_E_ARG, "qf_sector_prepare: null sector or state");
        if (occ_mask >> (2 * s->n_orb))
            return fail(QF_E_RANGE, "qf_sector_prepare: occ_mask has a bit >= 2 n_orb");
        const uint32_t ra = s->rankA[compact(occ_mask, 0, s->n_orb)], rb = s->rankB[compact(occ_mask, 1, s->n_orb)];
        if (ra == kNoRank || rb == kNoRank)
            return fail(QF_E_RANGE, "qf_sector_prepare: the reference is not in the sector");
        const uint64_t dim = (uint64_t)s->DA * s->DB;
        const unsigned nb = (unsigned)std::min<uint64_t>((dim + kBlock - 1) / kBlock, 8 * kMaxBlocks);
        hipLaunchKernelGGL(k_sector_prepare, dim3(nb), dim3(kBlock), 0, (hipStream_t)stream, (double2 *)psi, dim,
                           (uint64_t)ra * s->DB + rb);
        QF_HIP(hipGetLastError());
        return QF_OK;
    });
}

extern "C" int qf_sector_apply(qf_sector *s, void *psi, const double *t, int inverse, void *stream)
{
    return guarded([&]() -> int {
        if (!s || !psi || (!s->exc.empty() && !t))
            return fail(QF_E_ARG, "qf_sector_apply: null argument");
        const size_t E = s->exc.size();
        for (size_t i = 0; i < E; i++) {
            const size_t m = inverse ? E - 1 - i : i;
            const double tm = inverse ? -t[m] : t[m];
            const uint32_t nrows = s->row0[m + 1] - s->row0[m];
            if (nrows == 0)
                continue;  // no determinant of the sector is in the domain
            hipLaunchKernelGGL(k_sector_rotate, dim3(exc_grid(*s, m)), dim3(kSecT), 0, (hipStream_t)stream,
                               (double2 *)psi, s->d_strA, s->d_strB, s->d_rankA, s->d_rankB, s->d_rows + s->row0[m],
                               nrows, s->DB, s->exc[m], std::cos(tm), std::sin(tm));
        }
        QF_HIP(hipGetLastError());
        return QF_OK;
    });
}

extern "C" int qf_sector_energy(qf_sector *s, const void *psi, double *E_out, void *stream)
{
    return guarded([&]() -> int {
        if (!s || !psi || !E_out)
            return fail(QF_E_ARG, "qf_sector_energy: null argument");
        if (s->G == 0) {
            *E_out = 0.0;
            return QF_OK;
        }
        hipStream_t st = (hipStream_t)stream;
        hipLaunchKernelGGL(k_sector_energy, dim3(tile_grid(*s)), dim3(kSecT), 0, st, (const double2 *)psi, s->d_strA,
                           s->d_strB, s->d_rankA, s->d_rankB, s->DA, s->DB, s->d_groups, s->G, s->d_strs,
                           s->d_partials, s->d_counter, s->d_result);
        QF_HIP(hipGetLastError());
        QF_HIP(hipMemcpyAsync(E_out, s->d_result, sizeof(double), hipMemcpyDeviceToHost, st));
        QF_HIP(hipStreamSynchronize(st));
        return QF_OK;
    });
}

extern "C" int qf_sector_energy_grad(qf_sector *s, uint64_t occ_mask, const double *t, void *workspace,
                                     double *E_out, double *dE_dt, void *stream)
{
    return guarded([&]() -> int {
        if (!s || !workspace || !E_out || (!s->exc.empty() && (!t || !dE_dt)))
            return fail(QF_E_ARG, "qf_sector_energy_grad: null argument");
        if (s->G == 0)
            return fail(QF_E_ARG, "qf_sector_energy_grad: the sector has no Hamiltonian");
        hipStream_t st = (hipStream_t)stream;
        double2 *phi = (double2 *)workspace;
        double2 *lam = phi + (uint64_t)s->DA * s->DB;
        int rc = qf_sector_prepare(s, phi, occ_mask, stream);
        if (rc != QF_OK)
            return rc;
        rc = qf_sector_apply(s, phi, t, 0, stream);
        if (rc != QF_OK)
            return rc;
        const unsigned grid = tile_grid(*s);
        hipLaunchKernelGGL(k_sector_sigma, dim3(grid), dim3(kSecT), 0, st, (const double2 *)phi, lam, s->d_strA,
                           s->d_strB, s->d_rankA, s->d_rankB, s->DA, s->DB, s->d_groups, s->G, s->d_strs,
                           s->d_partials, s->d_counter, s->d_result);
        const size_t E = s->exc.size();
        if (E > s->grad_cap) {
            if (s->d_grad)
                QF_HIP(hipFree(s->d_grad));
            s->d_grad = nullptr;
            s->d_grad = dev_alloc<double>(E);
            s->grad_cap = E;
        }
        for (size_t i = E; i-- > 0;)
            hipLaunchKernelGGL(k_sector_adjoint, dim3(s->part0[i + 1] - s->part0[i]), dim3(kSecT), 0, st, phi, lam,
                               s->d_strA, s->d_strB, s->d_rankA, s->d_rankB, s->d_rows + s->row0[i],
                               s->row0[i + 1] - s->row0[i], s->DB, s->exc[i], std::cos(t[i]), std::sin(t[i]),
                               s->d_part + s->part0[i]);
        if (E)
            hipLaunchKernelGGL(k_sector_grad_reduce, dim3((unsigned)((E + kSecT - 1) / kSecT)), dim3(kSecT), 0, st,
                               s->d_part, s->d_part0, (int)E, s->d_grad);
        QF_HIP(hipGetLastError());
        QF_HIP(hipMemcpyAsync(E_out, s->d_result, sizeof(double), hipMemcpyDeviceToHost, st));
        if (E)
            QF_HIP(hipMemcpyAsync(dE_dt, s->d_grad, E * sizeof(double), hipMemcpyDeviceToHost, st));
        QF_HIP(hipStreamSynchronize(st));
        return QF_OK;
    });
}
