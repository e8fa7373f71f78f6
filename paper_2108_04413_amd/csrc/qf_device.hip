// Device side of the Pauli-exponential state-vector library (gfx950).
//
// State: 2^n complex128 amplitudes (double2), qubit q = bit q of the index.
// A Pauli string P(x, z) = i^popcount(x&z) X^x Z^z maps |y> to
// omega(y) |y ^ x>, omega(y) = i^(popcount(x&z) + 2 popcount(y&z)).
//
// Kernels (FP64 throughout):
//   k_prepare        one write pass: psi = |occ>.
//   k_run_tables     per fused run, cos/sin of the combined angle for each
//                    sign pattern (tiny).
//   k_apply_block    a segment of runs (flip masks inside one set Q of B
//                    qubits) applied to LDS sub-cubes of 2^B amplitudes:
//                    one HBM read and write of the state per segment (the
//                    ordered product of Sec. 2.1.4 exponentials, fused).
//   k_apply_run /    one pass per run too wide for a sub-cube: every pair
//   k_apply_diag     (y, y^x) gets one 2x2 rotation (a phase if x = 0).
//   k_energy_stream  <psi|H|psi> over tiles of 2^11 amplitudes: groups whose
//                    flip masks agree above bit 11 form a class, one state
//                    read per class, strings merged per tile (Sec. 3.1,
//                    Eq. (17)), work items interleaved over the classes;
//                    k_energy_tiled / k_energy_merged walk the same items
//                    class by class (per string / merged), k_energy makes
//                    one pass per group.
//   k_sigma_stream   lambda = H psi over output tiles of 2^11: per class the
//                    partner tile staged in LDS, strings merged per tile into
//                    lo-terms with signs taken at the output index, fused
//                    with E = Re <psi|lambda>; k_sigma gathers psi[y ^ x_g]
//                    per group below 12 qubits.
//   k_adjoint_block  reverse sweep over a segment on LDS sub-cubes of phi and
//                    lambda: 2 Im <lambda|P_k|phi> for each string of a run,
//                    then phi, lambda <- U_run^dagger; k_grad_reduce adds
//                    the per-workgroup string sums; k_adjoint_run is the
//                    one-run form.
// Reductions are deterministic: per-block partials in a fixed shape, then
// the last block to finish (ticket counter) sums them in index order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "qf_common.h"
#include "qf_kernels.h"
#include "qf_host.h"

namespace qf {

// Block-wide deterministic sum of M values per thread, then the last block
// to arrive sums the per-block partials in block order into out[0..M).
template <int M, int NTH = kBlock>
__device__ void reduce_finish(double (&v)[M], double *partials, unsigned *counter, double *out,
                              double scale, int nout)
{
    __shared__ double lds[NTH / 64][M];
    __shared__ bool last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < M; k++) {
        double s = v[k];
        for (int off = 32; off > 0; off >>= 1)
            s += __shfl_xor(s, off, 64);
        if (lane == 0)
            lds[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
        for (int w = 0; w < NTH / 64; w++)
            s += lds[w][threadIdx.x];
        __hip_atomic_store(&partials[(size_t)blockIdx.x * M + threadIdx.x], s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    // fixed-shape tree: thread t sums blocks t, t + NTH, ... for each k
    const int nb = gridDim.x;
    __shared__ double red[NTH];
    for (int k = 0; k < M; k++) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += NTH)
            s += __hip_atomic_load(&partials[(size_t)b * M + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = NTH / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0 && k < nout)
            out[k] = scale * red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ kernels

__global__ __launch_bounds__(kBlock) void k_prepare(double2 *__restrict__ psi, uint64_t dim, uint32_t occ)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t y = (uint64_t)blockIdx.x * kBlock + threadIdx.x; y < dim; y += stride)
        psi[y] = make_double2(y == occ ? 1.0 : 0.0, 0.0);
}

// <a|x_j> and <b|x_j> for the J <= JMAX states x_j = xs + j * dim: out[2j],
// out[2j + 1] the real and imaginary parts of <a|x_j>, out[2 JMAX + 2j],
// out[2 JMAX + 2j + 1] those of <b|x_j>; fixed-order reduction.
constexpr int kMaxDots = 16;
template <int JMAX>
__global__ __launch_bounds__(kBlock) void k_dots(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                 const double2 *__restrict__ xs, uint64_t dim, int J,
                                                 double *partials, unsigned *counter, double *out)
{
    double v[4 * JMAX];
#pragma unroll
    for (int k = 0; k < 4 * JMAX; k++)
        v[k] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t y = (uint64_t)blockIdx.x * kBlock + threadIdx.x; y < dim; y += stride) {
        const double2 av = a[y], bv = b[y];
#pragma unroll
        for (int j = 0; j < JMAX; j++) {
            if (j < J) {
                const double2 x = xs[(uint64_t)j * dim + y];
                v[2 * j] += av.x * x.x + av.y * x.y;
                v[2 * j + 1] += av.x * x.y - av.y * x.x;
                v[2 * JMAX + 2 * j] += bv.x * x.x + bv.y * x.y;
                v[2 * JMAX + 2 * j + 1] += bv.x * x.y - bv.y * x.x;
            }
        }
    }
    reduce_finish<4 * JMAX>(v, partials, counter, out, 1.0, 4 * JMAX);
}

// out[i] = psi[idx[i]]: the amplitudes at a list of basis states.
__global__ __launch_bounds__(kBlock) void k_gather(const double2 *__restrict__ psi, const uint64_t *__restrict__ idx,
                                                   int64_t count, double2 *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        out[i] = psi[idx[i]];
}

__global__ __launch_bounds__(64) void k_zero_u32(unsigned *__restrict__ p, unsigned count)
{
    for (unsigned i = threadIdx.x; i < count; i += blockDim.x)
        p[i] = 0u;
}

// One block per run; Theta(u) = sum_k s_k (-1)^popcount(u & e_k) theta_k.
__global__ __launch_bounds__(64) void k_run_tables(const RunDesc *__restrict__ runs,
                                                   const double *__restrict__ theta,
                                                   double2 *__restrict__ tab)
{
    const RunDesc d = runs[blockIdx.x];
    for (int u = threadIdx.x; u < (1 << d.r); u += blockDim.x) {
        double th = 0.0;
        for (int k = 0; k < d.m; k++) {
            const double v = (double)d.s[k] * theta[d.k0 + k];
            th += (__popc((uint32_t)u & d.e[k]) & 1) ? -v : v;
        }
        double sn, cs;
        sincos(th, &sn, &cs);
        tab[d.tab + u] = make_double2(cs, sn);
    }
}

// psi <- U_run psi (sgn = +1) or U_run^dagger psi (sgn = -1), x != 0.
__global__ __launch_bounds__(kBlock) void k_apply_run(double2 *__restrict__ psi, uint64_t npairs,
                                                      RunDesc d, const double2 *__restrict__ tab,
                                                      double sgn)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kItems) + threadIdx.x;
    uint32_t y[kItems];
    double2 a[kItems], b[kItems];
    bool ok[kItems];
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const uint64_t j = base + (uint64_t)i * kBlock;
        ok[i] = j < npairs;
        y[i] = insert0((uint32_t)(ok[i] ? j : 0), d.hbit);
        if (ok[i]) {
            a[i] = psi[y[i]];
            b[i] = psi[y[i] ^ d.x];
        }
    }
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        if (!ok[i])
            continue;
        const uint32_t y1 = y[i], y2 = y1 ^ d.x;
        const double2 cs = tab[d.tab + run_coords(d, y1)];
        const double c = cs.x, s = sgn * cs.y;
        const double2 pb = mul_ik((d.a0 + 2u * par(y2 & d.z0)) & 3u, b[i]);  // (P0 psi)[y1]
        const double2 pa = mul_ik((d.a0 + 2u * par(y1 & d.z0)) & 3u, a[i]);  // (P0 psi)[y2]
        // new = c v - i s (p)  ->  (c v.x + s p.y, c v.y - s p.x)
        psi[y1] = make_double2(c * a[i].x + s * pb.y, c * a[i].y - s * pb.x);
        psi[y2] = make_double2(c * b[i].x + s * pa.y, c * b[i].y - s * pa.x);
    }
}

// Pairs of one flip run on a sub-cube in LDS.  Thread t's items are pair
// indices t + k * NT (k < NP); y1 = insert0(j, hbit) has its table index and
// Z-parity split into the thread's part (ut, pt31) and item k's part (the
// run's item table).  pt31 carries, in bit 31, the Z-parity of y_t plus the
// constant signs of the rotation; px31 the parity of x & z0.
// All items are read before any is written: the pairs are disjoint, but the
// compiler cannot tell, and item by item it would wait out one LDS round
// trip per item.
template <bool SW, uint32_t NB, int NT>
__device__ __forceinline__ void apply_pairs(double2 *st, const double2 *tb, const LocalRun &d, uint32_t yt,
                                            uint32_t ut, uint32_t pt31, uint32_t px31)
{
    constexpr int NP = NB / 2 >= (uint32_t)NT ? (int)(NB / 2 / NT) : 1;
    if (NB / 2 < (uint32_t)NT && threadIdx.x >= NB / 2)
        return;
    uint32_t y1[NP];
    double2 a[NP], b[NP], cs[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const uint32_t ik = item_part(item_table(d), k);
        y1[k] = yt | insert0((uint32_t)k * NT, d.hbit);
        cs[k] = tb[ut ^ (ik & 63u)];
        a[k] = st[y1[k]];
        b[k] = st[y1[k] ^ d.x];
    }
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const uint32_t P1 = pt31 ^ ((item_part(item_table(d), k) >> 6) << 31);
        rot_pair<SW>(cs[k].x, flip31(cs[k].y, P1), flip31(cs[k].y, P1 ^ px31), a[k], b[k]);
        st[y1[k]] = a[k];
        st[y1[k] ^ d.x] = b[k];
    }
}

// Blocked apply: one workgroup per sub-cube of 2^B amplitudes.  Runs of the
// segment are applied in order (or reversed, with sgn = -1, for U^dagger);
// the pairs (y, y ^ x) of a run never leave the sub-cube because x is in Q.
// The segment's (cos, sin) tables are staged in LDS with the sub-cube, and
// so are the parities of the sub-cube's fixed bits against every run.
template <int B, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_apply_block(
    double2 *__restrict__ psi, Segment sg, const LocalRun *__restrict__ lruns,
    const ApplyTriple *__restrict__ trip, const double2 *__restrict__ tab, double sgn)
{
    constexpr uint32_t NB = 1u << B;
    static_assert(NT <= (int)NB && NB % NT == 0, "the workgroup must tile the sub-cube");
    constexpr int PER = (int)(NB / NT);
    static_assert(PER == 1 || NT == kItemStride, "a thread's items are kItemStride apart");
    __shared__ double2 st[NB];
    __shared__ uint32_t hoff[kMaxHoff];
    __shared__ double2 stab[kSegTab];
    __shared__ uint32_t spbz[kSegRuns];
    // base: the block index scattered into the qubits outside Q
    const uint32_t base = subcube_base(blockIdx.x, sg);
    const uint32_t lomask = (1u << sg.q0) - 1u;
    if (threadIdx.x < (1u << sg.nhi)) {
        uint32_t o = 0;
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (q < sg.nhi)
                o |= ((threadIdx.x >> q) & 1u) << sg.hi[q];
        hoff[threadIdx.x] = o;
    }
    for (int t = threadIdx.x; t < sg.ntab; t += NT)
        stab[t] = tab[sg.tab0 + t];
    const int nr = sg.r1 - sg.r0;
    sub_parities(lruns, sg.r0, nr, base, spbz, (int)threadIdx.x, NT);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const uint32_t l = threadIdx.x + (uint32_t)i * NT;
        st[l] = psi[base | (l & lomask) | hoff[l >> sg.q0]];
    }
    const uint32_t sneg = sgn < 0 ? 1u : 0u;
    // three runs per pass need a coset of 8 amplitudes per thread (trip is
    // read only then)
    constexpr bool kThree = NB == 8u * (uint32_t)NT;
    for (int ri = 0; ri < nr; ri++) {
        const int rr = sgn > 0 ? ri : nr - 1 - ri;
        const LocalRun d = lruns[sg.r0 + rr];
        if constexpr (kThree) {
            // a flip run's itm[1] is free: it carries the triple flags
            if (d.x && (d.itm[1] & (sneg ? 2u : 1u))) {
                const int r0 = sneg ? rr - 2 : rr;
                const ApplyTriple T = trip[sg.r0 + r0];
                __syncthreads();
                if (sneg)
                    apply_three<false>(st, stab, T, spbz + r0, threadIdx.x);
                else
                    apply_three<true>(st, stab, T, spbz + r0, threadIdx.x);
                ri += 2;
                continue;
            }
        }
        const double2 *tb = stab + (d.tab - sg.tab0);
        const uint32_t pbz = spbz[rr];
        __syncthreads();
        if (d.x) {
            // a' = c a - i sgn s i^k2 b with i^k2 = i^a0 (-1)^p2, so the
            // rotation factor is sgn (-1)^p2 i^m, m = a0 + 3
            const uint32_t m = (d.a0 + 3u) & 3u;
            const uint32_t yt = insert0(threadIdx.x, d.hbit);
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(yt, d.b, d.r);
            const uint32_t pt31 = (par(yt & d.z0) ^ (pbz >> 6) ^ (m >> 1) ^ sneg) << 31;
            const uint32_t px31 = par(d.x & d.z0) << 31;
            if (m & 1u)
                apply_pairs<true, NB, NT>(st, tb, d, yt, ut, pt31, px31);
            else
                apply_pairs<false, NB, NT>(st, tb, d, yt, ut, pt31, px31);
        } else {
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(threadIdx.x, d.b, d.r);
            double2 cs[PER], v[PER];
#pragma unroll
            for (int k = 0; k < PER; k++) {
                cs[k] = tb[ut ^ item_part(item_table(d), k)];
                v[k] = st[threadIdx.x + (uint32_t)k * NT];
            }
#pragma unroll
            for (int k = 0; k < PER; k++) {
                const double c = cs[k].x, s = sgn * cs[k].y;
                st[threadIdx.x + (uint32_t)k * NT] = make_double2(c * v[k].x + s * v[k].y, c * v[k].y - s * v[k].x);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; i++) {
        uint32_t l = threadIdx.x + (uint32_t)i * NT;
        // (an empty register barrier: the write-back forms its addresses
        // again instead of keeping those of the loads live through the run
        // loop, where they would spill)
        asm volatile("" : "+v"(l));
        psi[base | (l & lomask) | hoff[l >> sg.q0]] = st[l];
    }
}

// Diagonal run (x == 0): psi[y] *= cos(Theta) - i sgn sin(Theta).
__global__ __launch_bounds__(kBlock) void k_apply_diag(double2 *__restrict__ psi, uint64_t dim, RunDesc d,
                                                       const double2 *__restrict__ tab, double sgn)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < dim; j += stride) {
        const uint32_t y = (uint32_t)j;
        const double2 cs = tab[d.tab + run_coords(d, y)];
        const double c = cs.x, s = sgn * cs.y;
        const double2 v = psi[y];
        psi[y] = make_double2(c * v.x + s * v.y, c * v.y - s * v.x);
    }
}

// E = sum_g sum_pairs 2 Re conj(psi[y^x]) D_g(y) psi[y]  (x != 0)
//   + sum_y |psi[y]|^2 D_0(y)                            (x == 0)
__global__ __launch_bounds__(kBlock) void k_energy(const double2 *__restrict__ psi, int n,
                                                   const GroupDesc *__restrict__ groups, int G,
                                                   const uint32_t *__restrict__ zs,
                                                   const double *__restrict__ cs, double *partials,
                                                   unsigned *counter, double *result)
{
    double acc = 0.0;
    for (int gi = 0; gi < G; gi++) {
        const GroupDesc g = groups[gi];
        const uint64_t npairs = g.x ? (1ull << (n - 1)) : (1ull << n);
        const uint64_t per = (uint64_t)kBlock * kItems;
        const uint64_t chunk = ((npairs + (uint64_t)gridDim.x * per - 1) / ((uint64_t)gridDim.x * per)) * per;
        const uint64_t start = (uint64_t)blockIdx.x * chunk;
        const uint64_t end = start + chunk < npairs ? start + chunk : npairs;
        const double w = g.x ? 2.0 : 1.0;
        for (uint64_t j0 = start + threadIdx.x; j0 < end; j0 += per) {
            uint32_t y[kItems];
            double2 a[kItems], b[kItems];
            bool ok[kItems];
#pragma unroll
            for (int i = 0; i < kItems; i++) {
                const uint64_t j = j0 + (uint64_t)i * kBlock;
                ok[i] = j < end;
                const uint32_t jj = (uint32_t)(ok[i] ? j : start);
                y[i] = g.x ? insert0(jj, g.hbit) : jj;
                a[i] = psi[y[i]];
                b[i] = psi[y[i] ^ g.x];
            }
            double dre[kItems], dim[kItems];
            group_d(g, zs, cs, y, dre, dim);
#pragma unroll
            for (int i = 0; i < kItems; i++) {
                const double tr = dre[i] * a[i].x - dim[i] * a[i].y;
                const double ti = dre[i] * a[i].y + dim[i] * a[i].x;
                const double v = b[i].x * tr + b[i].y * ti;
                acc += ok[i] ? w * v : 0.0;
            }
        }
    }
    double vals[1] = {acc};
    reduce_finish<1>(vals, partials, counter, result, 1.0, 1);
}

// Tiled energy: tiles of 2^LT amplitudes; a work item is (class c, tile t1)
// with partner tile t2 = t1 ^ xh_c.  The partner tile is staged in LDS and
// every group of the class is evaluated on the item, so the state is read
// once per class instead of once per group.  For xh != 0 the own tile has
// bit hb of its index clear and each pair (y in t1, y ^ x in t2) counts twice
// (2 Re); for xh == 0 the partner of y is in the same tile and the sum runs
// over every y with weight 1 (sum_y conj(psi[y^x]) D(y) psi[y] = <P_g>).
template <int LT>
__global__ __launch_bounds__(kBlock) void k_energy_tiled(const double2 *__restrict__ psi,
                                                         const ClassDesc *__restrict__ classes,
                                                         const uint64_t *__restrict__ work_off,
                                                         uint64_t total_work,
                                                         const GroupDesc *__restrict__ groups,
                                                         const uint32_t *__restrict__ zs,
                                                         const double *__restrict__ cs, double *partials,
                                                         unsigned *counter, double *result)
{
    constexpr uint32_t T = 1u << LT;
    constexpr int kChunk = kBlock * kItems;
    __shared__ double2 tile[T];
    double acc = 0.0;
    int c = 0;
    for (uint64_t w = blockIdx.x; w < total_work; w += gridDim.x) {
        while (w >= work_off[c + 1])
            c++;
        const ClassDesc cd = classes[c];
        const uint32_t j = (uint32_t)(w - work_off[c]);
        const uint32_t t1 = cd.xh ? insert0(j, cd.hb) : j;
        const uint32_t t2 = t1 ^ cd.xh;
        const double wt = cd.xh ? 2.0 : 1.0;
        __syncthreads();  // the previous item's LDS reads are done
        const double2 *src = psi + ((size_t)t2 << LT);
#pragma unroll 4
        for (uint32_t i = threadIdx.x; i < T; i += kBlock)
            tile[i] = src[i];
        __syncthreads();
        const double2 *own = psi + ((size_t)t1 << LT);
        for (uint32_t base = 0; base < T; base += kChunk) {
            uint32_t ylo[kItems], y[kItems];
            double2 a[kItems];
#pragma unroll
            for (int i = 0; i < kItems; i++) {
                ylo[i] = base + threadIdx.x + (uint32_t)i * kBlock;
                y[i] = (t1 << LT) | ylo[i];
            }
            if (cd.xh) {
#pragma unroll
                for (int i = 0; i < kItems; i++)
                    a[i] = own[ylo[i]];
            } else {
#pragma unroll
                for (int i = 0; i < kItems; i++)
                    a[i] = tile[ylo[i]];
            }
            for (int gi = cd.g0; gi < cd.g1; gi++) {
                const GroupDesc g = groups[gi];
                const uint32_t xl = g.x & (T - 1u);
                double2 b[kItems];
#pragma unroll
                for (int i = 0; i < kItems; i++)
                    b[i] = tile[ylo[i] ^ xl];
                double dre[kItems], dim[kItems];
                group_d(g, zs, cs, y, dre, dim);
#pragma unroll
                for (int i = 0; i < kItems; i++) {
                    const double tr = dre[i] * a[i].x - dim[i] * a[i].y;
                    const double ti = dre[i] * a[i].y + dim[i] * a[i].x;
                    acc += wt * (b[i].x * tr + b[i].y * ti);
                }
            }
        }
    }
    double vals[1] = {acc};
    reduce_finish<1>(vals, partials, counter, result, 1.0, 1);
}

// Merged tiled energy (same schedule as k_energy_tiled).  Group descriptors
// index string records: [k0, kre) real phase, [kre, k1) imaginary phase.
// Per work item the coefficient of a lo-term, sum_k c_k (-1)^popcount(t1 & zhi_k),
// is uniform across the block; each own amplitude then needs one parity and
// one FMA with +-1.0 per lo-term.  Own amplitudes are processed NI at a time.
template <int NI>
__device__ __forceinline__ void apply_lo_terms(const ERec *__restrict__ recs, int r0, int r1, uint32_t t1,
                                               const uint32_t (&ylo)[NI], double (&sg)[NI], double (&d)[NI])
{
    if (r0 >= r1)
        return;
    double ce = 0.0;
    ERec e = recs[r0];
    for (int r = r0; r < r1; r++) {
        const ERec en = recs[r + 1 < r1 ? r + 1 : r];  // prefetch
        ce += flip(e.c, par(t1 & e.zhi));
        if (e.emit) {
#pragma unroll
            for (int i = 0; i < NI; i++) {
                sg[i] = __hiloint2double((int)(0x3FF00000u | (__popc(ylo[i] & e.zlo) << 31)), __double2loint(sg[i]));
                d[i] = fma(sg[i], ce, d[i]);
            }
            ce = 0.0;
        }
        e = en;
    }
}

template <int LT, int NI>
__global__ __launch_bounds__(kBlock) void k_energy_merged(const double2 *__restrict__ psi,
                                                          const ClassDesc *__restrict__ classes,
                                                          const uint64_t *__restrict__ work_off,
                                                          uint64_t total_work,
                                                          const GroupDesc *__restrict__ groups,
                                                          const ERec *__restrict__ recs, double *partials,
                                                          unsigned *counter, double *result)
{
    constexpr uint32_t T = 1u << LT;
    constexpr uint32_t kChunk = (uint32_t)kBlock * NI;
    static_assert(T % kChunk == 0, "tile must be a multiple of the chunk");
    __shared__ double2 tile[T];
    double acc = 0.0;
    double sg[NI];  // +-1.0: only the high word changes
#pragma unroll
    for (int i = 0; i < NI; i++)
        sg[i] = 1.0;
    int c = 0;
    for (uint64_t w = blockIdx.x; w < total_work; w += gridDim.x) {
        while (w >= work_off[c + 1])
            c++;
        const ClassDesc cd = classes[c];
        const uint32_t j = (uint32_t)(w - work_off[c]);
        const uint32_t t1 = cd.xh ? insert0(j, cd.hb) : j;
        const uint32_t t2 = t1 ^ cd.xh;
        const double wt = cd.xh ? 2.0 : 1.0;
        __syncthreads();
        const double2 *src = psi + ((size_t)t2 << LT);
#pragma unroll 4
        for (uint32_t i = threadIdx.x; i < T; i += kBlock)
            tile[i] = src[i];
        __syncthreads();
        const double2 *own = psi + ((size_t)t1 << LT);
        for (uint32_t base = 0; base < T; base += kChunk) {
            uint32_t ylo[NI];
            double2 a[NI];
#pragma unroll
            for (int i = 0; i < NI; i++)
                ylo[i] = base + threadIdx.x + (uint32_t)i * kBlock;
            if (cd.xh) {  // uniform branch: global loads, or LDS when the pair is in one tile
#pragma unroll
                for (int i = 0; i < NI; i++)
                    a[i] = own[ylo[i]];
            } else {
#pragma unroll
                for (int i = 0; i < NI; i++)
                    a[i] = tile[ylo[i]];
            }
            for (int gi = cd.g0; gi < cd.g1; gi++) {
                const GroupDesc g = groups[gi];
                const uint32_t xl = g.x & (T - 1u);
                double2 b[NI];
#pragma unroll
                for (int i = 0; i < NI; i++)
                    b[i] = tile[ylo[i] ^ xl];
                double dre[NI], dim[NI];
#pragma unroll
                for (int i = 0; i < NI; i++) {
                    dre[i] = 0.0;
                    dim[i] = 0.0;
                }
                apply_lo_terms<NI>(recs, g.k0, g.kre, t1, ylo, sg, dre);
                apply_lo_terms<NI>(recs, g.kre, g.k1, t1, ylo, sg, dim);
#pragma unroll
                for (int i = 0; i < NI; i++) {
                    const double tr = dre[i] * a[i].x - dim[i] * a[i].y;
                    const double ti = dre[i] * a[i].y + dim[i] * a[i].x;
                    acc += wt * (b[i].x * tr + b[i].y * ti);
                }
            }
        }
    }
    double vals[1] = {acc};
    reduce_finish<1>(vals, partials, counter, result, 1.0, 1);
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Streaming form of the merged 2^11-tile energy.  Work items follow the
// interleaved piece order, and the descriptor of the item after the fetched
// one is read a step ahead.  The fetch of an item also loads one of its group
// descriptors and one of its records per thread; at the item's start these go
// to LDS beside the partner tile, and every wave then pulls them 64 at a time
// into registers and broadcasts them with readlane.  Vector loads that the
// compute waits for are therefore always older than the next item's tile
// loads, which stay in flight during the compute.  Items with more than 256
// groups or records restage the rest from global memory.
//
// With y_lo = tid + 256 i, the lo-term sign (-1)^popcount(y_lo & z_lo) splits
// into a per-thread factor (bits 0..7 of z_lo) and a wave-uniform factor per
// element slot i (bits 8..10), so an element costs one FMA per lo-term.
template <bool IMAG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_energy_stream(const double2 *__restrict__ psi,
                                                          const VClass *__restrict__ vcls, uint32_t nv,
                                                          uint32_t per_v, const GroupDesc *__restrict__ groups,
                                                          const ERec *__restrict__ recs, double *partials,
                                                          unsigned *counter, double *result)
{
    constexpr int LT = 11;
    constexpr int NI = 8;
    constexpr uint32_t T = 1u << LT;
    constexpr int W = kBlock;  // staged groups / records per window
    static_assert(T == (uint32_t)kBlock * NI, "one tile per block pass");
    static_assert(NI == 8, "slot i of a thread is bits 8..10 of y_lo");
    __shared__ double2 tile[T];
    __shared__ uint4 sgrp[W];  // x & (T-1), kre, k1
    __shared__ uint4 srec[W];  // z_lo | emit << 31, z_hi, c (lo, hi word)
    const uint32_t tid = threadIdx.x;
    const int lane = (int)(tid & 63u);
    double acc = 0.0;

    auto load_group = [&](int gi) __attribute__((always_inline)) {
        const GroupDesc g = groups[gi];
        return make_uint4(g.x & (T - 1u), (uint32_t)g.kre, (uint32_t)g.k1, g.x >> 31);
    };
    auto load_rec = [&](int ri) __attribute__((always_inline)) {
        const ERec e = recs[ri];
        return make_uint4(e.zlo | (e.emit << 31), e.zhi, (uint32_t)__double2loint(e.c),
                          (uint32_t)__double2hiint(e.c));
    };

    // items in order (p, round): piece vcls[p] at tile pair vcls[p].j0 + round
    const uint32_t dp = gridDim.x % nv, dj = gridDim.x / nv;
    uint32_t pf = blockIdx.x % nv, jf = blockIdx.x / nv;  // the item to fetch next
    bool hf = jf < per_v;
    VClass vf = vcls[hf ? pf : 0u];  // nv >= 1: a valid piece even for an idle block
    VClass vc = vf;                  // the item whose data is in flight
    bool hc = false;

    double2 pn[NI], on[NI];  // partner and own tile of the fetched item
    // one group and one record of it, raw: no arithmetic on loaded values
    // before the next item's start, so the fetch never waits on its loads
    uint32_t qg_x = 0, qg_re = 0, qg_end = 0, qr_zlo = 0, qr_emit = 0, qr_zhi = 0;
    double qr_c = 0.0;
    uint32_t t1n = 0;
#pragma unroll
    for (int i = 0; i < NI; i++) {
        pn[i] = make_double2(0.0, 0.0);
        on[i] = pn[i];
    }

    while (hc || hf) {
        uint32_t p3 = pf + dp, j3 = jf + dj;
        if (p3 >= nv) {
            p3 -= nv;
            j3++;
        }
        const bool h3 = hf && j3 < per_v;
        const VClass v3 = vcls[h3 ? p3 : pf];

        const uint32_t t1 = t1n;
        double2 a[NI];
        if (hc) {
            __syncthreads();  // the previous item's LDS reads are done
#pragma unroll
            for (int i = 0; i < NI; i++) {
                tile[tid + (uint32_t)i * kBlock] = pn[i];
                a[i] = on[i];
            }
            sgrp[tid] = make_uint4(qg_x & (T - 1u), qg_re, qg_end, qg_x >> 31);
            srec[tid] = make_uint4(qr_zlo | (qr_emit << 31), qr_zhi, (uint32_t)__double2loint(qr_c),
                                   (uint32_t)__double2hiint(qr_c));
            __syncthreads();
        }
        {
            // unconditional, so the in-flight registers need no merge copies
            // (a copy would wait on the loads); past the end this re-reads
            // the last valid tile pair of the piece
            const uint32_t j = vf.j0 + min(jf, per_v - 1u);
            const uint32_t t1f = vf.xh ? insert0(j, vf.hb) : j;
            const double2 *q2 = psi + ((size_t)(t1f ^ vf.xh) << LT);
            const double2 *q1 = psi + ((size_t)t1f << LT);
#pragma unroll
            for (int i = 0; i < NI; i++)
                pn[i] = q2[tid + (uint32_t)i * kBlock];
#pragma unroll
            for (int i = 0; i < NI; i++)
                on[i] = q1[tid + (uint32_t)i * kBlock];
            {
                const GroupDesc &g = groups[min(vf.g0 + (int)tid, vf.g1 - 1)];
                qg_x = g.x;
                qg_re = (uint32_t)g.kre;
                qg_end = (uint32_t)g.k1;
                const ERec &e = recs[min(vf.r0 + (int)tid, vf.r1 - 1)];
                qr_zlo = e.zlo;
                qr_emit = e.emit;
                qr_zhi = e.zhi;
                qr_c = e.c;
            }
            t1n = t1f;
        }
        if (hc) {
            // ---- record cursor: chunk [rc, rc + 64) of the item's records, one
            // per lane; cv holds the segmented prefix sums of the signed
            // coefficients (segments end at lo-term emits), so at an emit lane
            // it is that lo-term's coefficient for this tile pair
            int wr = vc.r0, rc = vc.r0 - 64;
            uint64_t emask = 0;
            uint32_t cz = 0;
            double cv = 0.0;
            auto prep = [&]() __attribute__((always_inline)) {
                double cin = 0.0;  // open lo-term carried from the previous chunk
                if (rc >= vc.r0) {
                    const uint32_t z63 = (uint32_t)__builtin_amdgcn_readlane((int)cz, 63);
                    cin = (z63 >> 31) ? 0.0 : readlane_d(cv, 63);
                }
                rc += 64;
                if (rc - wr == W) {
                    __syncthreads();
                    srec[tid] = load_rec(min(rc + (int)tid, vc.r1 - 1));
                    wr = rc;
                    __syncthreads();
                }
                const uint4 e = srec[rc - wr + lane];
                const bool valid = rc + lane < vc.r1;
                const uint32_t z = valid ? e.x : 0u;
                double sv = valid ? flip(__hiloint2double((int)e.w, (int)e.z), par(t1 & e.y)) : 0.0;
                const uint64_t em = __ballot((z >> 31) != 0u);
                // segment start: lane 0 or the lane after an emit
                int sf = lane == 0 || ((em >> (lane - 1)) & 1ull);
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const double up = __shfl_up(sv, (unsigned)off, 64);
                    const int upf = __shfl_up(sf, (unsigned)off, 64);
                    if (lane >= off) {
                        if (!sf)
                            sv += up;
                        sf |= upf;
                    }
                }
                const int first = em ? __builtin_ctzll(em) : 63;
                if (lane <= first)
                    sv += cin;
                emask = em;
                cz = z;
                cv = sv;
            };
            int r = vc.r0;  // next record to consume
            auto next_lo = [&](uint32_t &z, double &ce) __attribute__((always_inline)) {
                while (emask == 0)
                    prep();
                const int k = __builtin_ctzll(emask);
                emask &= emask - 1;
                z = (uint32_t)__builtin_amdgcn_readlane((int)cz, k);
                ce = readlane_d(cv, k);
                r = rc + k + 1;
            };

            // lo-terms of one phase part, up to record rend, into d[i].  Slot
            // i's sign is (-1)^popcount(i & K), K = bits 8..10 of z_lo, and
            // the lo-terms (sorted by z_lo) come in runs of equal K: a run
            // sums a = sum s0 ce once, then adds (-1)^popcount(i & K) a to
            // the eight slots (uniform signs from an XOR table of K's bits)
            auto part = [&](int rend, double(&d)[NI]) __attribute__((always_inline)) {
                double a = 0.0;
                uint32_t Kc = 8u;  // no run open
                auto flush = [&]() __attribute__((always_inline)) {
                    const uint32_t c1 = Kc << 31, c2 = (Kc >> 1) << 31, c4 = (Kc >> 2) << 31;
                    const uint32_t sk[NI] = {0u, c1, c2, c1 ^ c2, c4, c1 ^ c4, c2 ^ c4, c1 ^ c2 ^ c4};
#pragma unroll
                    for (int i = 0; i < NI; i++)
                        d[i] = fma(pm_one(sk[i]), a, d[i]);
                };
                while (r < rend) {
                    uint32_t z;
                    double ce;
                    next_lo(z, ce);
                    const uint32_t zl = z & (T - 1u);
                    const uint32_t K = zl >> 8;
                    if (K != Kc) {
                        if (Kc < 8u)
                            flush();
                        a = 0.0;
                        Kc = K;
                    }
                    a = fma(pm_one((uint32_t)__popc(tid & zl) << 31), ce, a);
                }
                if (Kc < 8u)
                    flush();
            };

            double item = 0.0;
            int wg = vc.g0, gc = vc.g0;
            uint4 gch = sgrp[lane];
            for (int gi = vc.g0; gi < vc.g1; gi++) {
                if (gi - gc == 64) {
                    gc = gi;
                    if (gc - wg == W) {
                        __syncthreads();
                        sgrp[tid] = load_group(min(gc + (int)tid, vc.g1 - 1));
                        wg = gc;
                        __syncthreads();
                    }
                    gch = sgrp[gc - wg + lane];
                }
                const int k = gi - gc;
                const uint32_t xl = (uint32_t)__builtin_amdgcn_readlane((int)gch.x, k);
                const int kre = __builtin_amdgcn_readlane((int)gch.y, k);
                const int k1 = __builtin_amdgcn_readlane((int)gch.z, k);
                if (!IMAG && __builtin_amdgcn_readlane((int)gch.w, k)) {
                    // one run (real part, one slot pattern K): the group adds
                    // a sum_i (-1)^popcount(i & K) Re(conj(b_i) a_i)
                    double sa = 0.0;
                    uint32_t K = 0u;
                    while (r < kre) {
                        uint32_t z;
                        double ce;
                        next_lo(z, ce);
                        const uint32_t zl = z & (T - 1u);
                        K = zl >> 8;
                        sa = fma(pm_one((uint32_t)__popc(tid & zl) << 31), ce, sa);
                    }
                    const uint32_t c1 = K << 31, c2 = (K >> 1) << 31, c4 = (K >> 2) << 31;
                    const uint32_t sk[NI] = {0u, c1, c2, c1 ^ c2, c4, c1 ^ c4, c2 ^ c4, c1 ^ c2 ^ c4};
                    double Q = 0.0;
#pragma unroll
                    for (int i = 0; i < NI; i++) {
                        const double2 b = tile[(tid + (uint32_t)i * kBlock) ^ xl];
                        Q = fma(pm_one(sk[i]), b.x * a[i].x + b.y * a[i].y, Q);
                    }
                    item = fma(sa, Q, item);
                    continue;
                }
                double dre[NI];
#pragma unroll
                for (int i = 0; i < NI; i++)
                    dre[i] = 0.0;
                part(kre, dre);
                if (IMAG) {
                    double dim[NI];
#pragma unroll
                    for (int i = 0; i < NI; i++)
                        dim[i] = 0.0;
                    part(k1, dim);
#pragma unroll
                    for (int i = 0; i < NI; i++) {
                        const double2 b = tile[(tid + (uint32_t)i * kBlock) ^ xl];
                        const double tr = dre[i] * a[i].x - dim[i] * a[i].y;
                        const double ti = dre[i] * a[i].y + dim[i] * a[i].x;
                        item += b.x * tr + b.y * ti;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < NI; i++) {
                        const double2 b = tile[(tid + (uint32_t)i * kBlock) ^ xl];
                        item = fma(dre[i], b.x * a[i].x + b.y * a[i].y, item);
                    }
                }
            }
            acc += (vc.xh ? 2.0 : 1.0) * item;
        }
        vc = vf;
        hc = hf;
        vf = v3;
        pf = p3;
        jf = j3;
        hf = h3;
    }
    double vals[1] = {acc};
    reduce_finish<1>(vals, partials, counter, result, 1.0, 1);
}

// lambda[y] = sum_g D_g(y ^ x_g) psi[y ^ x_g];  E = Re sum_y conj(psi[y]) lambda[y]
__global__ __launch_bounds__(kBlock) void k_sigma(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                                  int n, const GroupDesc *__restrict__ groups, int G,
                                                  const uint32_t *__restrict__ zs,
                                                  const double *__restrict__ cs, double *partials,
                                                  unsigned *counter, double *result)
{
    const uint64_t dim = 1ull << n;
    const uint64_t per = (uint64_t)kBlock * kItems;
    double acc = 0.0;
    for (uint64_t j0 = (uint64_t)blockIdx.x * per; j0 < dim; j0 += (uint64_t)gridDim.x * per) {
        uint32_t y[kItems];
        bool ok[kItems];
        double2 l[kItems];
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t j = j0 + threadIdx.x + (uint64_t)i * kBlock;
            ok[i] = j < dim;
            y[i] = (uint32_t)(ok[i] ? j : 0);
            l[i] = make_double2(0.0, 0.0);
        }
        // Two groups at a time: both groups' gathers are issued first, so
        // the second group's loads are in flight while the first group's
        // coefficients are evaluated (the pass is bound by gathers from
        // L2 / Infinity Cache).
        static_assert(kItems == 4 && kBlock == 256, "items are y0 + 256 i, i < 4");
        const uint32_t yt = (uint32_t)(j0 + threadIdx.x);
        auto gather = [&](const GroupDesc &g, double2 (&b)[kItems]) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < kItems; i++)
                b[i] = psi[y[i] ^ g.x];
        };
        auto add_group = [&](const GroupDesc &g, const double2 (&b)[kItems]) __attribute__((always_inline)) {
            double dre[kItems], dimg[kItems];
            group_d4<8>(g, zs, cs, yt ^ g.x, dre, dimg);
#pragma unroll
            for (int i = 0; i < kItems; i++) {
                l[i].x += dre[i] * b[i].x - dimg[i] * b[i].y;
                l[i].y += dre[i] * b[i].y + dimg[i] * b[i].x;
            }
        };
        for (int gi = 0; gi < G; gi += 2) {
            const bool two = gi + 1 < G;
            const GroupDesc ga = groups[gi], gb = groups[two ? gi + 1 : gi];
            double2 ba[kItems], bb[kItems];
            gather(ga, ba);
            gather(gb, bb);
            add_group(ga, ba);
            if (two)
                add_group(gb, bb);
        }
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            if (!ok[i])
                continue;
            lam[y[i]] = l[i];
            const double2 p = psi[y[i]];
            acc += p.x * l[i].x + p.y * l[i].y;
        }
    }
    double vals[1] = {acc};
    reduce_finish<1>(vals, partials, counter, result, 1.0, 1);
}

// lambda = H psi by the streamed tile routine (sigma_stream): one output tile
// of 2^11 per workgroup at a time, 256 threads of eight items.
constexpr int kSsNT = 256;

template <bool IMAG>
__device__ __forceinline__ void sigma_stream_kernel(const double2 *__restrict__ psi, double2 *__restrict__ lam, int n,
                                                    const SsCls *__restrict__ cls, int ncls,
                                                    const uint32_t *__restrict__ gwords, const SsLo *__restrict__ los,
                                                    double *partials, unsigned *counter, double *result)
{
    __shared__ double2 tile[1u << kSsL];
    __shared__ uint4 wlo[kSsNT];    // z_lo | flags, 0, C (lo, hi word)
    __shared__ uint32_t wgw[kSsNT]; // x & (2^11 - 1) | one-run pattern | lo-term count << 16
    double vals[1] = {sigma_stream<kSsNT, IMAG>(psi, lam, blockIdx.x, gridDim.x, 1u << (n - kSsL), cls, ncls,
                                                gwords, los, tile, wlo, wgw)};
    reduce_finish<1, kSsNT>(vals, partials, counter, result, 1.0, 1);
}

template <bool IMAG>
__global__ __launch_bounds__(kSsNT) void k_sigma_stream(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                                        int n, const SsCls *__restrict__ cls, int ncls,
                                                        const uint32_t *__restrict__ gwords,
                                                        const SsLo *__restrict__ los, double *partials,
                                                        unsigned *counter, double *result)
{
    sigma_stream_kernel<IMAG>(psi, lam, n, cls, ncls, gwords, los, partials, counter, result);
}

// Real phases only: held to 128 registers, four waves per SIMD (the LDS
// image admits four workgroups per CU; at 132 registers only three fit; the
// bound spills one 8-byte value per tile, outside the group loop).
template <>
__global__ __launch_bounds__(kSsNT) __attribute__((amdgpu_waves_per_eu(4))) void k_sigma_stream<false>(
    const double2 *__restrict__ psi, double2 *__restrict__ lam, int n, const SsCls *__restrict__ cls, int ncls,
    const uint32_t *__restrict__ gwords, const SsLo *__restrict__ los, double *partials, unsigned *counter,
    double *result)
{
    sigma_stream_kernel<false>(psi, lam, n, cls, ncls, gwords, los, partials, counter, result);
}

// One reverse-sweep step over a run: grad[k0+k] = 2 Im <lam|P_k|phi>, then
// phi, lam <- U_run^dagger (phi, lam).
__global__ __launch_bounds__(kBlock) void k_adjoint_run(double2 *__restrict__ phi, double2 *__restrict__ lam,
                                                        uint64_t npairs, RunDesc d,
                                                        const double2 *__restrict__ tab, double *partials,
                                                        unsigned *counter, double *grad)
{
    double acc[kMaxRun];
#pragma unroll
    for (int k = 0; k < kMaxRun; k++)
        acc[k] = 0.0;
    const uint64_t per = (uint64_t)kBlock * kItems;
    const bool diag = d.x == 0;
    for (uint64_t j0 = (uint64_t)blockIdx.x * per; j0 < npairs; j0 += (uint64_t)gridDim.x * per) {
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t j = j0 + threadIdx.x + (uint64_t)i * kBlock;
            if (j >= npairs)
                break;
            const uint32_t y1 = diag ? (uint32_t)j : insert0((uint32_t)j, d.hbit);
            const uint32_t y2 = y1 ^ d.x;
            const double2 a = phi[y1], la = lam[y1];
            const uint32_t u = run_coords(d, y1);
            const double2 cs = tab[d.tab + u];
            const double c = cs.x, s = cs.y;
            double q;
            if (diag) {
                // Im conj(la) a
                q = la.x * a.y - la.y * a.x;
                // U^dagger: v * (c + i s)
                phi[y1] = make_double2(c * a.x - s * a.y, c * a.y + s * a.x);
                lam[y1] = make_double2(c * la.x - s * la.y, c * la.y + s * la.x);
            } else {
                const double2 b = phi[y2], lb = lam[y2];
                const uint32_t k1 = (d.a0 + 2u * par(y1 & d.z0)) & 3u;
                const uint32_t k2 = (d.a0 + 2u * par(y2 & d.z0)) & 3u;
                const double2 wa = mul_ik(k1, a), wb = mul_ik(k2, b);
                // Q = conj(lb) wa + conj(la) wb ; q = Im Q
                q = (lb.x * wa.y - lb.y * wa.x) + (la.x * wb.y - la.y * wb.x);
                // U^dagger: new = c v + i s p -> (c v.x - s p.y, c v.y + s p.x)
                phi[y1] = make_double2(c * a.x - s * wb.y, c * a.y + s * wb.x);
                phi[y2] = make_double2(c * b.x - s * wa.y, c * b.y + s * wa.x);
                const double2 wla = mul_ik(k1, la), wlb = mul_ik(k2, lb);
                lam[y1] = make_double2(c * la.x - s * wlb.y, c * la.y + s * wlb.x);
                lam[y2] = make_double2(c * lb.x - s * wla.y, c * lb.y + s * wla.x);
            }
#pragma unroll
            for (int k = 0; k < kMaxRun; k++) {
                const double v = flip((double)d.s[k] * q, __popc(u & d.e[k]) & 1u);
                acc[k] += k < d.m ? v : 0.0;
            }
        }
    }
    reduce_finish<kMaxRun>(acc, partials, counter, grad + d.k0, 2.0, d.m);
}


// Blocked reverse sweep over one segment of runs: each workgroup holds one
// 2^B sub-cube of phi and of lambda in LDS and walks the segment's runs in
// reverse; for each run it first accumulates 2 Im <lambda|P_k|phi> of the
// run's strings over the sub-cube (before the run is undone), then undoes the
// run on both states.  The grid is persistent (resident workgroups, each
// looping over sub-cubes) and keeps per-string sums in LDS; the last
// workgroup to finish sums the per-workgroup sums in workgroup order.
constexpr int adj_threads(int B) { return B >= 10 ? 512 : (1 << B) / 2 >= 256 ? 256 : 64; }

// Pairs of one flip run in the reverse sweep (items as in apply_pairs).
// Before the run is undone, q = 2 Im <lambda|P_0|phi> / 2 over the pair with
// P_0's phase i^a0 (-1)^p split off: q = Im[i^a0 ((-1)^p1 conj(lb) a +
// (-1)^p2 conj(la) b)], which is the imaginary part (a0 even) or the real
// part (a0 odd) of the bracket, negated for a0 >= 2.  Undoing the run is
// rot_pair with the factor (-1)^p i^(a0 + 1); SW = (a0 + 1) & 1, so SW also
// selects Im.  dq31 is the sign of q relative to the rotation's signs.  The
// items' q go to accumulate(u_0, du, q) together (du[k] = u_0 ^ u_k, the
// same for every thread).
// UNDO = false only accumulates (the pool-gradient sweep: nothing is undone).
template <bool SW, uint32_t NB, int NT, bool UNDO, class Acc>
__device__ __forceinline__ void adjoint_pairs(double2 *sp, double2 *sl, const double2 *tb, const LocalRun &d,
                                              uint32_t yt, uint32_t ut, uint32_t pt31, uint32_t px31,
                                              uint32_t dq31, Acc &&accumulate)
{
    constexpr int NP = NB / 2 >= (uint32_t)NT ? (int)(NB / 2 / NT) : 1;
    if (NB / 2 < (uint32_t)NT && threadIdx.x >= NB / 2)
        return;
    const uint32_t i0 = item_part(item_table(d), 0) & 63u;
    uint32_t du[NP], y1s[NP];
    double qs[NP];
    double2 as[NP], bs[NP], las[NP], lbs[NP], css[NP];
    // every item is read before any is written (the pairs are disjoint; item
    // by item the compiler would wait out one LDS round trip per item)
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const uint32_t ik = item_part(item_table(d), k);
        const uint32_t y1 = yt | insert0((uint32_t)k * NT, d.hbit), y2 = y1 ^ d.x;
        y1s[k] = y1;
        if constexpr (UNDO)
            css[k] = tb[ut ^ (ik & 63u)];
        as[k] = sp[y1];
        bs[k] = sp[y2];
        las[k] = sl[y1];
        lbs[k] = sl[y2];
    }
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const uint32_t ik = item_part(item_table(d), k);
        const uint32_t y1 = y1s[k], y2 = y1 ^ d.x;
        du[k] = i0 ^ (ik & 63u);
        const uint32_t P1 = pt31 ^ ((ik >> 6) << 31), P2 = P1 ^ px31;
        double2 a = as[k], b = bs[k], la = las[k], lb = lbs[k];
        const double f1 = SW ? lb.x * a.y - lb.y * a.x : lb.x * a.x + lb.y * a.y;
        const double f2 = SW ? la.x * b.y - la.y * b.x : la.x * b.x + la.y * b.y;
        const double q = flip31(f1, P1 ^ dq31) + flip31(f2, P2 ^ dq31);
        if constexpr (UNDO) {
            const double2 cs = css[k];
            const double s1 = flip31(cs.y, P1), s2 = flip31(cs.y, P2);
            rot_pair<SW>(cs.x, s1, s2, a, b);
            rot_pair<SW>(cs.x, s1, s2, la, lb);
            sp[y1] = a;
            sp[y2] = b;
            sl[y1] = la;
            sl[y2] = lb;
        }
        qs[k] = q;
    }
    accumulate(ut ^ i0, du, qs);
}

// UNDO = false: the same string sums 2 Im <lambda|P_k|phi> with phi and
// lambda left as they are (read-only sub-cubes, no write-back): the ADAPT
// pool gradients of Sec. 3.2 on a fixed state.
template <int B, int NT, bool UNDO = true>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_adjoint_block(double2 *__restrict__ phi, double2 *__restrict__ lam, int n,
                                                      Segment sg, const LocalRun *__restrict__ lruns,
                                                      const AdjPair *__restrict__ apairs,
                                                      const uint32_t *__restrict__ smap,
                                                      const double2 *__restrict__ tab, int sk0, int nstr,
                                                      double *__restrict__ part, int K)
{
    constexpr uint32_t NB = 1u << B;
    static_assert(NT <= (int)NB && NB % NT == 0 && NT % 64 == 0, "the workgroup must tile the sub-cube");
    constexpr int PER = (int)(NB / NT);
    constexpr int NW = NT / 64;
    __shared__ double2 sp[NB], sl[NB];
    __shared__ uint32_t hoff[kMaxHoff];
    // runs per segment: the read-only sweep stages no tables, which leaves
    // room for the sums of more runs
    constexpr int RMAX = UNDO ? kAdjRuns : kPoolRuns;
    __shared__ double2 stab[UNDO ? kAdjTab : 1];
    // per wave and run, the run's 8 sums over this workgroup's sub-cubes so
    // far (each wave adds to its own: no barrier, no cross-wave step per run)
    __shared__ double wred[NW][RMAX][kMaxRun];
    __shared__ uint32_t spbz[RMAX];
    static_assert(PER == 1 || NT == kItemStride, "a thread's items are kItemStride apart");
    // two runs per pass need a coset of 4 amplitudes per thread (apairs is
    // read only then)
    constexpr bool kTwo = UNDO && NB == 4u * (uint32_t)NT;
    const uint32_t tid = threadIdx.x;
    const int lane = (int)(tid & 63u), wave = (int)(tid >> 6);
    const uint32_t lomask = (1u << sg.q0) - 1u;
    if (tid < (1u << sg.nhi)) {
        uint32_t o = 0;
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (q < sg.nhi)
                o |= ((tid >> q) & 1u) << sg.hi[q];
        hoff[tid] = o;
    }
    if constexpr (UNDO)
        for (int t = (int)tid; t < sg.ntab; t += NT)
            stab[t] = tab[sg.tab0 + t];
    for (int t = (int)tid; t < NW * RMAX * kMaxRun; t += NT)
        (&wred[0][0][0])[t] = 0.0;
    const uint32_t nsub = 1u << (n - B);
    const int nr = sg.r1 - sg.r0;
    // thread r < nr keeps run r's full-space masks (z0f, bf) in registers for
    // the per-sub-cube parities (nr <= RMAX < NT)
    uint32_t pm[kMaxRank + 1] = {};
    if (tid < (uint32_t)nr) {
        const LocalRun &d = lruns[sg.r0 + (int)tid];
        pm[kMaxRank] = d.z0f;
#pragma unroll
        for (int q = 0; q < kMaxRank; q++)
            pm[q] = d.bf[q];
    }
    for (uint32_t sc = blockIdx.x; sc < nsub; sc += gridDim.x) {
        const uint32_t base = subcube_base(sc, sg);
        // (the previous sub-cube's runs have all read spbz: barrier before its write-back)
        if (tid < (uint32_t)nr) {
            uint32_t v = par(base & pm[kMaxRank]) << 6;
#pragma unroll
            for (int q = 0; q < kMaxRank; q++)
                v |= par(base & pm[q]) << q;
            spbz[tid] = v;
        }
        __syncthreads();  // tables staged; the previous sub-cube is written back
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const uint32_t l = tid + (uint32_t)i * NT;
            const uint32_t y = base | (l & lomask) | hoff[l >> sg.q0];
            sp[l] = phi[y];
            sl[l] = lam[y];
        }
        if constexpr (!UNDO)
            __syncthreads();  // the sub-cube is loaded (the undo path waits at every run)
        for (int ri = nr - 1; ri >= 0; ri--) {
            if constexpr (kTwo) {
                const AdjPair pr = apairs[sg.r0 + ri];
                if (pr.w0 & 1u) {
                    const uint32_t pbzA = spbz[ri], pbzB = spbz[ri - 1];
                    __syncthreads();  // the previous run's updates are visible
                    adjoint_two<true>(sp, sl, stab, pr, pbzA, pbzB, tid, lane, wred[wave][ri], wred[wave][ri - 1]);
                    ri--;
                    continue;
                }
            }
            // (the descriptors stay in the scalar cache over the sub-cubes of
            // a segment; reading them a run ahead cost ~60 register copies per run)
            const LocalRun d = lruns[sg.r0 + ri];
            const double2 *tb = stab + (d.tab - sg.tab0);
            const uint32_t pbz = spbz[ri];
            // string k's weight is eps_k = s_k (-1)^popcount(u & e_k) with
            // s_k = +-1 and e_k < 2^r.  For r <= 3 the pass accumulates the 8
            // Walsh sums W[e] = sum (-1)^popcount(u & e) q (acc[e]) and string
            // k takes s_k W[e_k] afterwards; for r > 3, acc[k] is string k's sum.
            const bool walsh = d.r <= 3;
            double acc[kMaxRun];
#pragma unroll
            for (int k = 0; k < kMaxRun; k++)
                acc[k] = -0.0;  // -0.0 + x is x, so the first term needs no add
            // items k of the thread have table indices u0 ^ du[k] (du uniform)
            auto accumulate = [&](uint32_t u0, const auto &du, const auto &q) __attribute__((always_inline)) {
                constexpr int N = (int)(sizeof(q) / sizeof(double));
                if (walsh) {
                    walsh_add<N>(acc, u0, du, q);
                } else {
#pragma unroll
                    for (int i = 0; i < N; i++)
#pragma unroll
                        for (int k = 0; k < kMaxRun; k++)
                            acc[k] += flip(q[i], (__popc((u0 ^ du[i]) & d.e[k]) ^ (d.s[k] < 0 ? 1u : 0u)) & 1u);
                }
            };
            // the previous run's updates are visible (read-only: nothing changes
            // between the runs of a sub-cube, and no barrier is needed)
            if constexpr (UNDO)
                __syncthreads();
            if (d.x) {
                const uint32_t m = (d.a0 + 1u) & 3u;
                const uint32_t yt = insert0(tid, d.hbit);
                const uint32_t ut = (pbz & 63u) ^ gf2_coords(yt, d.b, d.r);
                const uint32_t pt31 = (par(yt & d.z0) ^ (pbz >> 6) ^ (m >> 1)) << 31;
                const uint32_t px31 = par(d.x & d.z0) << 31;
                const uint32_t dq31 = ((d.a0 >> 1) ^ (m >> 1)) << 31;
                if (m & 1u)
                    adjoint_pairs<true, NB, NT, UNDO>(sp, sl, tb, d, yt, ut, pt31, px31, dq31, accumulate);
                else
                    adjoint_pairs<false, NB, NT, UNDO>(sp, sl, tb, d, yt, ut, pt31, px31, dq31, accumulate);
            } else {
                const uint32_t ut = (pbz & 63u) ^ gf2_coords(tid, d.b, d.r);
                const uint32_t i0 = item_part(item_table(d), 0);
                uint32_t du[PER];
                double qs[PER];
                double2 as[PER], las[PER], css[PER];
#pragma unroll
                for (int kk = 0; kk < PER; kk++) {
                    const uint32_t y = tid + (uint32_t)kk * NT;
                    if constexpr (UNDO)
                        css[kk] = tb[ut ^ item_part(item_table(d), kk)];
                    as[kk] = sp[y];
                    las[kk] = sl[y];
                }
#pragma unroll
                for (int kk = 0; kk < PER; kk++) {
                    const uint32_t y = tid + (uint32_t)kk * NT;
                    du[kk] = i0 ^ item_part(item_table(d), kk);
                    const double2 a = as[kk], la = las[kk];
                    qs[kk] = la.x * a.y - la.y * a.x;
                    if constexpr (UNDO) {
                        const double c = css[kk].x, s = css[kk].y;
                        sp[y] = make_double2(c * a.x - s * a.y, c * a.y + s * a.x);
                        sl[y] = make_double2(c * la.x - s * la.y, c * la.y + s * la.x);
                    }
                }
                accumulate(ut ^ i0, du, qs);
            }
            {
                const double h = wave_sum8(acc, lane);
                if (sum8_writer(lane))
                    wave_add(&wred[wave][ri][sum8_index(lane)], h);
            }
        }
        __syncthreads();
        if constexpr (UNDO) {
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const uint32_t l = tid + (uint32_t)i * NT;
                const uint32_t y = base | (l & lomask) | hoff[l >> sg.q0];
                phi[y] = sp[l];
                lam[y] = sl[l];
            }
        }
    }
    // this workgroup's string sums, the waves added in order: string k of
    // run r takes s_k times Walsh sum e_k (rank <= 3) or sum k.  k_grad_reduce
    // adds the workgroups after the sweep (no cross-workgroup fence here: on
    // a multi-XCD device a release at agent scope writes back the whole L2,
    // sub-cube stores included)
    // (smap: the run, column and sign of each string, per string of the plan)
    __syncthreads();
    for (int t = (int)tid; t < nstr; t += NT) {
        const uint32_t e = smap[sk0 + t];
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++)
            v += wred[w][e >> 4][e & 7u];
        part[(size_t)blockIdx.x * K + sk0 + t] = (e & 8u) ? -v : v;
    }
}

// grad[k] = 2 sum_b part[b][k] in workgroup order, for the strings of
// blocked segments: 64 strings per workgroup (one per lane), the four waves
// split the workgroup range with 4 loads in flight each.
__global__ __launch_bounds__(kBlock) void k_grad_reduce(const double *__restrict__ part, int nb, int K,
                                                        const uint8_t *__restrict__ blocked, double *grad)
{
    __shared__ double ws[kBlock / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kBlock / 64;
    const int k = blockIdx.x * 64 + lane;
    double v = 0.0;
    if (k < K) {
        int b = wave;
        for (; b + 3 * NW < nb; b += 4 * NW) {
            double t[4];
#pragma unroll
            for (int u = 0; u < 4; u++)
                t[u] = part[(size_t)(b + u * NW) * K + k];
#pragma unroll
            for (int u = 0; u < 4; u++)
                v += t[u];
        }
        for (; b < nb; b += NW)
            v += part[(size_t)b * K + k];
    }
    ws[wave][lane] = v;
    __syncthreads();
    if (wave == 0 && k < K && blocked[k]) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++)
            t += ws[w][lane];
        grad[k] = 2.0 * t;
    }
}
} // namespace qf

// ===================================================================== host

namespace qf {

void check_terms(const char *who, int n, const qf_term *t, int64_t K)
{
    const uint64_t lim = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (int64_t k = 0; k < K; k++)
        if ((t[k].x & ~lim) || (t[k].z & ~lim))
            raise(QF_E_RANGE, std::string(who) + ": term " + std::to_string(k) + " has a mask bit >= n_qubits");
}

// Split a term list into fused runs: consecutive strings with the same flip
// mask whose Y-parity agrees (so they commute), at most kMaxRun strings and
// a sign-pattern space of rank <= kMaxRank.
std::vector<RunDesc> make_runs(const qf_term *T, int64_t K, int &tab_entries)
{
    std::vector<RunDesc> runs;
    tab_entries = 0;
    int64_t k = 0;
    while (k < K) {
        RunDesc d;
        std::memset(&d, 0, sizeof d);
        const uint32_t x = (uint32_t)T[k].x;
        const uint32_t zf = (uint32_t)T[k].z;
        const int afull = popc64(T[k].x & T[k].z);
        d.x = x;
        d.z0 = x ? zf : 0u;
        d.a0 = x ? (uint32_t)(afull & 3) : 0u;
        d.hbit = hibit(x);
        d.k0 = (int32_t)k;
        uint32_t rv[kMaxRank], cm[kMaxRank];
        int piv[kMaxRank];
        int r = 0, m = 0;
        while (k < K && m < kMaxRun && (uint32_t)T[k].x == x) {
            const int ak = popc64(T[k].x & T[k].z);
            if (((ak - afull) & 1) != 0)
                break;  // anticommutes with the run
            const uint32_t dv = x ? ((uint32_t)T[k].z ^ d.z0) : (uint32_t)T[k].z;
            uint32_t v = dv, coords = 0;
            for (int i = 0; i < r; i++)
                if ((v >> piv[i]) & 1u) {
                    v ^= rv[i];
                    coords ^= cm[i];
                }
            if (v) {
                if (r == kMaxRank)
                    break;
                d.b[r] = dv;
                rv[r] = v;
                cm[r] = coords ^ (1u << r);
                piv[r] = (int)hibit(v);
                coords = 1u << r;
                r++;
            }
            d.e[m] = (uint8_t)coords;
            d.s[m] = x ? ((((ak - afull) & 3) == 0) ? 1 : -1) : 1;
            m++;
            k++;
        }
        d.r = r;
        d.m = m;
        d.tab = tab_entries;
        tab_entries += 1 << r;
        runs.push_back(d);
    }
    return runs;
}

// Host tables of a grouped Hamiltonian: per group, real-phase strings first,
// with the sign of i^popcount(x&z) folded into the coefficient.
void build_groups(int n, const qf_term *H, const int64_t *goff, int64_t G, std::vector<GroupDesc> &gd,
                  std::vector<uint32_t> &zs, std::vector<double> &cs)
{
    if (goff[0] != 0)
        raise(QF_E_ARG, "group_off[0] must be 0");
    const int64_t KH = goff[G];
    check_terms("hamiltonian", n, H, KH);
    gd.assign((size_t)G, GroupDesc{});
    zs.assign((size_t)KH, 0u);
    cs.assign((size_t)KH, 0.0);
    for (int64_t g = 0; g < G; g++) {
        const int64_t a = goff[g], b = goff[g + 1];
        if (b < a || b > KH)
            raise(QF_E_ARG, "group_off is not monotone");
        if (b == a)
            raise(QF_E_ARG, "empty group " + std::to_string(g));
        const uint64_t x = H[a].x;
        int64_t w = a;
        for (int pass = 0; pass < 2; pass++) {
            for (int64_t k = a; k < b; k++) {
                if (H[k].x != x)
                    raise(QF_E_ARG, "group " + std::to_string(g) + " mixes flip masks");
                const int ph = popc64(H[k].x & H[k].z) & 3;
                if ((ph & 1) != pass)
                    continue;
                zs[(size_t)w] = (uint32_t)H[k].z;
                cs[(size_t)w] = (ph & 2) ? -H[k].c : H[k].c;
                w++;
            }
            if (pass == 0)
                gd[(size_t)g].kre = (int32_t)w;
        }
        gd[(size_t)g].x = (uint32_t)x;
        gd[(size_t)g].hbit = hibit((uint32_t)x);
        gd[(size_t)g].k0 = (int32_t)a;
        gd[(size_t)g].k1 = (int32_t)b;
        // the item-sign pattern of each phase part (0xF: the strings differ)
        auto pattern = [&](int64_t k0, int64_t k1) {
            int p = -1;
            for (int64_t k = k0; k < k1; k++) {
                const int q = (int)((zs[(size_t)k] >> kPatBit) & 3u);
                if (p >= 0 && q != p)
                    return 15;
                p = q;
            }
            return p < 0 ? 0 : p;
        };
        gd[(size_t)g].pat = pattern(a, gd[(size_t)g].kre) | (pattern(gd[(size_t)g].kre, b) << 4);
    }
}

namespace {

uint32_t pext32(uint32_t v, uint32_t mask)
{
    uint32_t out = 0, k = 0;
    for (int p = 0; p < 32; p++)
        if ((mask >> p) & 1u) {
            out |= ((v >> p) & 1u) << k;
            k++;
        }
    return out;
}

} // namespace

// Tables of the streamed sigma (sigma_stream) for workgroups of nt threads
// (256 or 512; item pattern p = z_lo >> log2(nt)): groups in class order,
// each group part's strings sorted by (z_lo, z_hi) and merged into lo-terms
// of equal z_lo (at most three strings each; longer runs continue in the
// next lo-term), the imaginary part's coefficients negated (signs taken at
// the output index), a flush flag on the last lo-term of every run of equal
// p.  A group of more than kSsGrp lo-terms is cut into groups of the same
// flip mask; sub-classes hold at most nt groups and nt lo-terms.  Group
// words: x & (2^11 - 1), the one-run flag and pattern, the lo-term count.
void sigma_stream_tables(const std::vector<GroupDesc> &gd, const std::vector<uint32_t> &zs,
                         const std::vector<double> &cs, int nt, std::vector<SsCls> &cls,
                         std::vector<uint32_t> &words, std::vector<SsLo> &los)
{
    if (nt != 256 && nt != 512)
        raise(QF_E_ARG, "streamed sigma tables: 256 or 512 threads");
    const int ps = nt == 256 ? 8 : 9;
    constexpr uint32_t lomask = (1u << kSsL) - 1u;
    std::vector<size_t> order(gd.size());
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return (gd[a].x >> kSsL) < (gd[b].x >> kSsL); });
    cls.clear();
    words.clear();
    los.clear();
    for (size_t gi : order) {
        const GroupDesc &g = gd[gi];
        std::vector<SsLo> lg;
        const int32_t ranges[2][2] = {{g.k0, g.kre}, {g.kre, g.k1}};
        for (int part = 0; part < 2; part++) {
            std::vector<int32_t> ks;
            for (int32_t k = ranges[part][0]; k < ranges[part][1]; k++)
                ks.push_back(k);
            std::stable_sort(ks.begin(), ks.end(), [&](int32_t a, int32_t b) {
                const uint32_t la = zs[(size_t)a] & lomask, lb = zs[(size_t)b] & lomask;
                return la != lb ? la < lb : (zs[(size_t)a] >> kSsL) < (zs[(size_t)b] >> kSsL);
            });
            const size_t first = lg.size();
            int used = 3;
            for (size_t i = 0; i < ks.size(); i++) {
                const uint32_t z = zs[(size_t)ks[i]];
                const uint32_t zlo = z & lomask;
                if (used == 3 || (lg.back().zf & lomask) != zlo) {
                    SsLo e;
                    std::memset(&e, 0, sizeof e);
                    e.zf = zlo | (part ? kSsImag : 0u);
                    lg.push_back(e);
                    used = 0;
                }
                lg.back().zhi[used] = z >> kSsL;
                lg.back().c[used] = part ? -cs[(size_t)ks[i]] : cs[(size_t)ks[i]];
                used++;
            }
            for (size_t j = first; j < lg.size(); j++)
                if (j + 1 == lg.size() || ((lg[j + 1].zf & lomask) >> ps) != ((lg[j].zf & lomask) >> ps))
                    lg[j].zf |= kSsFlush;
        }
        for (size_t p0 = 0; p0 < lg.size(); p0 += kSsGrp) {
            const size_t p1 = std::min(lg.size(), p0 + (size_t)kSsGrp);
            lg[p1 - 1].zf |= kSsFlush;
            const uint32_t xh = g.x >> kSsL;
            const int32_t nl = (int32_t)(p1 - p0);
            if (cls.empty() || cls.back().xh != xh || cls.back().ng == nt || cls.back().nl + nl > nt) {
                SsCls c;
                std::memset(&c, 0, sizeof c);
                c.xh = xh;
                c.g0 = (int32_t)words.size();
                c.l0 = (int32_t)los.size();
                cls.push_back(c);
            }
            // one run: every lo-term of the piece is real with one item pattern
            bool one = true;
            for (size_t j = p0; j < p1; j++)
                one = one && !(lg[j].zf & kSsImag) && ((lg[j].zf & lomask) >> ps) == ((lg[p0].zf & lomask) >> ps);
            const uint32_t pat = one ? (((lg[p0].zf & lomask) >> ps) << 11) | kSsOne : 0u;
            words.push_back((g.x & lomask) | pat | ((uint32_t)nl << 16));
            los.insert(los.end(), lg.begin() + (ptrdiff_t)p0, lg.begin() + (ptrdiff_t)p1);
            cls.back().ng++;
            cls.back().nl += nl;
        }
    }
}

// Greedy segmentation of the run sequence for blocked application: extend a
// segment while the union of its flip masks and the lowest q0 qubits has at
// most B qubits, it has at most max_runs runs (max_runs > 0) and its tables
// at most max_tab entries; pad Q with the lowest free qubits to exactly B.  A
// run whose mask alone does not fit becomes a segment with Q = 0 (applied by
// itself).
void build_segments(const std::vector<RunDesc> &runs, int n, int B, int q0, std::vector<Segment> &segs,
                    std::vector<LocalRun> &lr, int max_runs, int max_tab)
{
    segs.clear();
    lr.clear();
    const uint32_t low = (1u << q0) - 1u;
    size_t i = 0;
    while (i < runs.size()) {
        uint32_t cur = low;
        size_t j = i;
        int ntab = 0;
        int nstr = 0;
        while (j < runs.size() && __builtin_popcount(cur | runs[j].x) <= B && ntab + (1 << runs[j].r) <= max_tab &&
               nstr + runs[j].m <= kSegStr && (max_runs == 0 || (int)(j - i) < max_runs)) {
            cur |= runs[j].x;
            ntab += 1 << runs[j].r;
            nstr += runs[j].m;
            j++;
        }
        Segment sg;
        std::memset(&sg, 0, sizeof sg);
        if (j == i) {  // does not fit a sub-cube
            sg.Q = 0;
            sg.r0 = (int32_t)i;
            sg.r1 = (int32_t)i + 1;
            segs.push_back(sg);
            i++;
            continue;
        }
        uint32_t Q = cur;
        for (int p = 0; p < n && __builtin_popcount(Q) < B; p++)
            Q |= 1u << p;
        int qlow = 0;
        while (qlow < 32 && ((Q >> qlow) & 1u))
            qlow++;
        if (B - qlow > 8)
            raise(QF_E_ARG, "segment: more than 8 sub-cube qubits above the contiguous rows");
        sg.Q = Q;
        sg.q0 = qlow;
        sg.nhi = 0;
        for (int p = qlow; p < n; p++)
            if ((Q >> p) & 1u)
                sg.hi[sg.nhi++] = (uint32_t)p;
        sg.r0 = (int32_t)lr.size();
        sg.tab0 = runs[i].tab;  // run tables are laid out in run order
        sg.ntab = runs[j - 1].tab + (1 << runs[j - 1].r) - runs[i].tab;
        for (size_t k = i; k < j; k++) {
            const RunDesc &d = runs[k];
            LocalRun L;
            std::memset(&L, 0, sizeof L);
            L.x = pext32(d.x, Q);
            L.hbit = hibit(L.x);
            L.z0 = pext32(d.z0, Q);
            L.a0 = d.a0;
            L.z0f = d.z0;
            for (int q = 0; q < d.r; q++) {
                L.b[q] = pext32(d.b[q], Q);
                L.bf[q] = d.b[q];
            }
            L.r = d.r;
            L.tab = d.tab;
            L.k0 = d.k0;
            L.m = d.m;
            for (int k = 0; k < kMaxRun; k++) {
                L.e[k] = d.e[k];
                L.s[k] = d.s[k];
            }
            // per-item parts of the table index and the Z-parity
            auto coords = [&](uint32_t y) {
                uint32_t u = 0;
                for (int q = 0; q < d.r; q++)
                    u |= (uint32_t)(__builtin_popcount(y & L.b[q]) & 1) << q;
                return u;
            };
            if (L.x) {
                for (int k = 0; k < 4; k++) {
                    const uint32_t j = (uint32_t)k * kItemStride;
                    const uint32_t lo = j & ((1u << L.hbit) - 1u);
                    const uint32_t yk = ((j ^ lo) << 1) | lo;
                    const uint32_t v = coords(yk) | (uint32_t)(__builtin_popcount(yk & L.z0) & 1) << 6;
                    L.itm[0] |= v << (8 * k);
                }
            } else {
                for (int k = 0; k < 8; k++)
                    L.itm[k >> 2] |= coords((uint32_t)k * kItemStride) << (8 * (k & 3));
            }
            lr.push_back(L);
        }
        sg.r1 = (int32_t)lr.size();
        segs.push_back(sg);
        i = j;
    }
}

// Two-run passes of the blocked reverse sweep (AdjPair): walking each
// segment's runs from the last, as the kernel does, run r and run r - 1 form
// a pair when both are flip runs of rank <= 3 with different flip masks and
// a0 odd; a run that does not pair is undone on its own.
std::vector<AdjPair> adjoint_pairs(const std::vector<Segment> &segs, const std::vector<LocalRun> &lr)
{
    std::vector<AdjPair> ap(lr.size());
    std::memset(ap.data(), 0, ap.size() * sizeof(AdjPair));
    auto par = [](uint32_t v) { return (uint32_t)__builtin_popcount(v) & 1u; };
    auto coords3 = [&](uint32_t y, const LocalRun &d) {
        return par(y & d.b[0]) | (par(y & d.b[1]) << 1) | (par(y & d.b[2]) << 2);
    };
    // bits 0..6 of one run: second-pair table offset, its parity offset,
    // par(x & z0), m >> 1 and the q sign (see AdjPair)
    auto run_bits = [&](const LocalRun &d, uint32_t other) {
        const uint32_t m = (d.a0 + 1u) & 3u;
        return coords3(other, d) | par(other & d.z0) << 3 | par(d.x & d.z0) << 4 | (m >> 1) << 5 |
               (((d.a0 >> 1) ^ (m >> 1)) & 1u) << 6;
    };
    for (const Segment &sg : segs) {
        if (!sg.Q)
            continue;
        for (int ri = sg.r1 - 1; ri >= sg.r0; ri--) {
            if (ri == sg.r0)
                break;
            const LocalRun &A = lr[(size_t)ri], &B = lr[(size_t)ri - 1];
            if (!(A.x && B.x && A.x != B.x && A.r <= 3 && B.r <= 3 && (A.a0 & B.a0 & 1u)))
                continue;
            const uint32_t p1 = A.hbit;
            const uint32_t xr = ((B.x >> p1) & 1u) ? B.x ^ A.x : B.x;
            const uint32_t p2 = 31u - (uint32_t)__builtin_clz(xr);
            AdjPair &P = ap[(size_t)ri];
            P.w0 = 1u | std::min(p1, p2) << 8 | std::max(p1, p2) << 16;
            P.xA = A.x;
            P.xB = B.x;
            for (int q = 0; q < 3; q++) {
                P.bA[q] = A.b[q];
                P.bB[q] = B.b[q];
            }
            P.z0A = A.z0;
            P.z0B = B.z0;
            P.bits = run_bits(A, B.x) | run_bits(B, A.x) << 8;
            P.tabs = (uint32_t)(A.tab - sg.tab0) | (uint32_t)(B.tab - sg.tab0) << 16;
            ri--;  // B is taken
        }
    }
    return ap;
}

// Three-run passes of the blocked apply (ApplyTriple), grouped greedily from
// each segment's first run.
std::vector<ApplyTriple> apply_triples(const std::vector<Segment> &segs, const std::vector<LocalRun> &lr)
{
    std::vector<ApplyTriple> at(lr.size());
    std::memset(at.data(), 0, at.size() * sizeof(ApplyTriple));
    auto par = [](uint32_t v) { return (uint32_t)__builtin_popcount(v) & 1u; };
    auto hib = [](uint32_t v) { return 31u - (uint32_t)__builtin_clz(v); };
    auto coords3 = [&](uint32_t y, const LocalRun &d) {
        return par(y & d.b[0]) | (par(y & d.b[1]) << 1) | (par(y & d.b[2]) << 2);
    };
    for (const Segment &sg : segs) {
        if (!sg.Q)
            continue;
        for (int ri = sg.r0; ri + 2 < sg.r1;) {
            const LocalRun *R[3] = {&lr[(size_t)ri], &lr[(size_t)ri + 1], &lr[(size_t)ri + 2]};
            bool ok = true;
            for (const LocalRun *d : R)
                ok = ok && d->x && d->r <= 3 && (d->a0 & 1u);
            uint32_t v0 = 0, v1 = 0, v2 = 0, p0 = 0, p1 = 0;
            if (ok) {
                v0 = R[0]->x;
                p0 = hib(v0);
                v1 = R[1]->x;
                if ((v1 >> p0) & 1u)
                    v1 ^= v0;
                ok = v1 != 0;
            }
            if (ok) {
                p1 = hib(v1);
                v2 = R[2]->x;
                if ((v2 >> p0) & 1u)
                    v2 ^= v0;
                if ((v2 >> p1) & 1u)
                    v2 ^= v1;
                ok = v2 != 0;
            }
            if (!ok) {
                ri++;
                continue;
            }
            uint32_t piv[3] = {p0, p1, hib(v2)};
            std::sort(piv, piv + 3);
            ApplyTriple &T = at[(size_t)ri];
            T.w0 = 1u | piv[0] << 8 | piv[1] << 16 | piv[2] << 24;
            for (int j = 0; j < 3; j++) {
                const LocalRun &d = *R[j];
                const int k1 = j == 0 ? 1 : 0, k2 = j == 2 ? 1 : 2;
                const uint32_t x1 = R[k1]->x, x2 = R[k2]->x;
                T.x[j] = d.x;
                for (int q = 0; q < 3; q++)
                    T.b[j][q] = d.b[q];
                T.z0[j] = d.z0;
                T.bits[j] = coords3(x1, d) | coords3(x2, d) << 3 | par(x1 & d.z0) << 6 | par(x2 & d.z0) << 7 |
                            par(d.x & d.z0) << 8 | (((d.a0 + 3u) & 3u) >> 1) << 9;
                T.tabs |= (uint32_t)(d.tab - sg.tab0) << (10 * j);
            }
            at[(size_t)ri + 2].w0 = 2u;
            ri += 3;
        }
    }
    return at;
}

} // namespace qf

struct qf_plan {
    int n = 0;
    int64_t K = 0;
    std::vector<qf::RunDesc> runs;
    int tab_entries = 0;
    qf::RunDesc *d_runs = nullptr;
    int block_bits = 0;                 // sub-cube size of blocked apply (0: per-run passes)
    std::vector<qf::Segment> segs;      // Q == 0: a run applied on its own (index r0)
    qf::LocalRun *d_lruns = nullptr;
    qf::ApplyTriple *d_atrip = nullptr;  // three-run passes of the blocked apply (2^12 sub-cubes), per LocalRun
    int adj_bits = 0;                   // sub-cube size of the blocked adjoint (0: per-run passes)
    std::vector<qf::Segment> asegs;     // segments of the blocked adjoint
    std::vector<int> aseg_k0, aseg_nstr; // their strings (contiguous: runs are in string order)
    qf::LocalRun *d_alruns = nullptr;
    qf::AdjPair *d_apairs = nullptr;    // two-run passes of the blocked adjoint, per LocalRun
    uint32_t *d_asmap = nullptr;        // per string of a blocked adjoint segment: run, Walsh column, sign
    double *d_apart = nullptr;          // per-block string sums of the blocked adjoint [adj_grid][K]
    uint8_t *d_ablocked = nullptr;      // 1 for strings of blocked adjoint segments
    unsigned adj_grid = 0;
    double *d_theta = nullptr;
    double *h_theta = nullptr;  // pinned staging for theta uploads
    hipEvent_t theta_done = nullptr;
    double2 *d_tab = nullptr;
    double *d_grad = nullptr;
    int G = 0;
    int tile_bits = 0;                 // 0: one pass per group; else tiled energy
    bool merged = false;               // tiled with per-item merged lo-terms
    bool has_imag = false;             // some Hamiltonian string has an odd number of Y
    qf::VClass *d_vcls = nullptr;      // 2^11 merged tiles: interleaved pieces of the streaming kernel
    uint32_t n_vcls = 0, per_vcls = 0;
    std::vector<qf::GroupDesc> groups; // host copies, for re-tiling
    std::vector<uint32_t> hz;
    std::vector<double> hc;
    qf::ERec *d_recs = nullptr;
    int64_t tiled_classes = 0;
    uint64_t tiled_work = 0;
    qf::ClassDesc *d_classes = nullptr;
    uint64_t *d_work_off = nullptr;
    qf::GroupDesc *d_tgroups = nullptr;
    qf::GroupDesc *d_groups = nullptr;
    uint32_t *d_z = nullptr;
    double *d_c = nullptr;
    qf::SsCls *d_ss_cls = nullptr;        // k_sigma_stream sub-classes, group words, lo-terms
    uint32_t *d_ss_words = nullptr;
    qf::SsLo *d_ss_los = nullptr;
    int n_ss_cls = 0;
    double *d_partials = nullptr;
    unsigned *d_counter = nullptr;
    double *d_result = nullptr;

    bool sigma_tables = true;             // build the sigma classes (not needed for energy only)

    // ADAPT pool plans (qf_plan_create_pool): the pool's strings are the
    // plan's "ansatz", members sorted by flip mask so that the blocked sweep
    // packs them into few segments; member i of the sorted order is caller
    // member pool_perm[i], its strings pool_off[i] .. pool_off[i + 1].
    std::vector<double> ac;      // the ansatz strings' coefficients (Trotter angles)
    double *d_dots = nullptr;    // QK: inner products of one state with a list of states
    uint64_t *d_pidx = nullptr;  // PQE: determinant indices to read (K entries)
    double2 *d_pout = nullptr;   // PQE: the amplitudes read there
    bool is_pool = false;
    std::vector<int64_t> pool_off, pool_perm;
    std::vector<double> pool_c;

    // Where the device arrays live.  kOwned: one hipMalloc per array, freed
    // with the plan.  kRegion: bump-allocated (256-byte aligned) from a
    // caller's region (an arena, or the library's static scratch), never
    // freed; uploads go through region_stream.  kMeasure: nothing touches
    // the device; region_used ends as the bytes a kRegion plan would need.
    enum Mem { kOwned, kRegion, kMeasure } mem = kOwned;
    char *region = nullptr;
    size_t region_cap = 0, region_used = 0;
    hipStream_t region_stream = nullptr;

    template <class T> T *dalloc(size_t count)
    {
        if (mem == kOwned)
            return qf::dev_alloc<T>(count);
        const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
        if (mem == kRegion && region_used + bytes > region_cap)
            qf::raise(QF_E_SIZE, "plan tables need more than the " + std::to_string(region_cap) +
                                     " bytes of the caller's region");
        // (a measuring plan hands out distinct non-null addresses that are never dereferenced)
        T *p = reinterpret_cast<T *>((mem == kRegion ? region : reinterpret_cast<char *>(256)) + region_used);
        region_used += bytes;
        return p;
    }
    void upload(void *dst, const void *src, size_t bytes)
    {
        if (mem == kMeasure || bytes == 0)
            return;
        if (mem == kOwned) {
            QF_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
            return;
        }
        // the host source is a temporary: wait for the copy before it goes
        QF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, region_stream));
        QF_HIP(hipStreamSynchronize(region_stream));
    }
    void release(void *p)
    {
        if (mem == kOwned && p)
            QF_HIP(hipFree(p));
    }

    ~qf_plan()
    {
        if (theta_done)
            (void)hipEventDestroy(theta_done);
        if (h_theta)
            (void)hipHostFree(h_theta);
        if (mem != kOwned)
            return;
        void *bufs[] = {d_runs, d_lruns, d_atrip, d_alruns, d_apairs, d_asmap, d_apart, d_ablocked, d_theta, d_tab, d_grad, d_groups, d_z, d_c, d_partials, d_counter, d_result,
                        d_classes, d_work_off, d_tgroups, d_recs, d_vcls, d_pidx, d_pout,
                        d_dots, d_ss_cls, d_ss_words, d_ss_los};
        for (void *p : bufs)
            if (p)
                (void)hipFree(p);
    }
};

namespace qf {

// Classes of groups sharing the flip bits above a tile of 2^L amplitudes,
// and the work-item offsets of the tiled energy kernel.
// Pieces of the streaming energy kernel, placed so that the costly ones
// (many records and groups per tile) are evenly spaced in every round.
void build_pieces(qf_plan &P, const std::vector<ClassDesc> &cls, const std::vector<GroupDesc> &tg)
{
    const uint32_t per = 1u << (P.n - 12);
    std::vector<VClass> pieces;
    std::vector<int64_t> cost;
    for (const ClassDesc &c : cls) {
        VClass v;
        std::memset(&v, 0, sizeof v);
        v.xh = c.xh;
        v.hb = c.hb;
        v.g0 = c.g0;
        v.g1 = c.g1;
        v.r0 = tg[(size_t)c.g0].k0;
        v.r1 = tg[(size_t)c.g1 - 1].k1;
        const int64_t w = (int64_t)(v.r1 - v.r0) + 2 * (int64_t)(v.g1 - v.g0);
        for (uint32_t h = 0; h < (c.xh ? 1u : 2u); h++) {
            v.j0 = h * per;
            pieces.push_back(v);
            cost.push_back(w);
        }
    }
    const uint32_t nv = (uint32_t)pieces.size();
    std::vector<VClass> placed(nv);
    std::vector<uint32_t> rank(nv);
    for (uint32_t i = 0; i < nv; i++)
        rank[i] = i;
    std::stable_sort(rank.begin(), rank.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
    // rank i goes to position i * stride mod nv: consecutive ranks land about
    // 0.618 nv apart, so every window of positions holds its share of costly pieces
    uint32_t stride = std::max<uint32_t>(1, (uint32_t)(0.6180339887 * nv));
    while (std::gcd(stride, nv) != 1)
        stride++;
    for (uint32_t i = 0; i < nv; i++)
        placed[(uint64_t)i * stride % nv] = pieces[rank[i]];
    P.d_vcls = P.dalloc<VClass>(nv);
    P.upload(P.d_vcls, placed.data(), nv * sizeof(VClass));
    P.n_vcls = nv;
    P.per_vcls = per;
}

void set_energy_tile(qf_plan &P, int L, bool merged)
{
    if (L != 0 && L != 10 && L != 11 && L != 12)
        raise(QF_E_ARG, "energy tile bits must be 0, 10, 11 or 12");
    if (L && P.n < L + 1)
        raise(QF_E_RANGE, "energy tile of 2^" + std::to_string(L) + " amplitudes needs n_qubits > " +
                              std::to_string(L));
    void *old[] = {P.d_classes, P.d_work_off, P.d_tgroups, P.d_recs, P.d_vcls};
    for (void *p : old)
        P.release(p);
    P.d_classes = nullptr;
    P.d_work_off = nullptr;
    P.d_tgroups = nullptr;
    P.d_recs = nullptr;
    P.d_vcls = nullptr;
    P.n_vcls = 0;
    P.per_vcls = 0;
    P.tile_bits = L;
    P.merged = L != 0 && merged;
    P.tiled_classes = 0;
    P.tiled_work = 0;
    if (!L || P.G == 0)
        return;
    std::vector<GroupDesc> tg(P.groups);
    std::stable_sort(tg.begin(), tg.end(),
                     [L](const GroupDesc &a, const GroupDesc &b) { return (a.x >> L) < (b.x >> L); });
    std::vector<ClassDesc> cls;
    std::vector<uint64_t> woff(1, 0);
    for (size_t g = 0; g < tg.size(); g++) {
        const uint32_t xh = tg[g].x >> L;
        if (cls.empty() || cls.back().xh != xh) {
            ClassDesc c;
            c.xh = xh;
            c.hb = hibit(xh);
            c.g0 = (int32_t)g;
            c.g1 = (int32_t)g;
            cls.push_back(c);
            woff.push_back(woff.back() + (xh ? (1ull << (P.n - L - 1)) : (1ull << (P.n - L))));
        }
        cls.back().g1 = (int32_t)g + 1;
    }
    if (P.merged) {
        // records of each phase part sorted by (z_lo, z_hi); the last record
        // of every run of equal z_lo closes a lo-term
        std::vector<ERec> recs;
        const uint32_t lomask = (1u << L) - 1u;
        for (GroupDesc &g : tg) {
            const int32_t ranges[2][2] = {{g.k0, g.kre}, {g.kre, g.k1}};
            GroupDesc ng = g;
            ng.k0 = (int32_t)recs.size();
            for (int part = 0; part < 2; part++) {
                std::vector<int32_t> ks;
                for (int32_t k = ranges[part][0]; k < ranges[part][1]; k++)
                    ks.push_back(k);
                std::stable_sort(ks.begin(), ks.end(), [&](int32_t a, int32_t b) {
                    const uint32_t la = P.hz[(size_t)a] & lomask, lb = P.hz[(size_t)b] & lomask;
                    return la != lb ? la < lb : (P.hz[(size_t)a] >> L) < (P.hz[(size_t)b] >> L);
                });
                for (size_t i = 0; i < ks.size(); i++) {
                    const uint32_t z = P.hz[(size_t)ks[i]];
                    ERec e;
                    std::memset(&e, 0, sizeof e);
                    e.zlo = z & lomask;
                    e.zhi = z >> L;
                    e.c = P.hc[(size_t)ks[i]];
                    e.emit = (i + 1 == ks.size() || (P.hz[(size_t)ks[i + 1]] & lomask) != e.zlo) ? 1u : 0u;
                    recs.push_back(e);
                }
                if (part == 0)
                    ng.kre = (int32_t)recs.size();
            }
            ng.k1 = (int32_t)recs.size();
            // bit 31 of x (n <= 30): one run for the streaming kernel (no
            // imaginary part, one slot pattern z_lo >> 8 over the records)
            if (L == 11 && ng.k1 == ng.kre && ng.k1 > ng.k0) {
                bool one = true;
                for (int32_t k = ng.k0; k < ng.k1; k++)
                    one = one && (recs[(size_t)k].zlo >> 8) == (recs[(size_t)ng.k0].zlo >> 8);
                if (one)
                    ng.x |= 0x80000000u;
            }
            g = ng;
        }
        P.d_recs = P.dalloc<ERec>(recs.size());
        P.upload(P.d_recs, recs.data(), recs.size() * sizeof(ERec));
        if (L == 11)
            build_pieces(P, cls, tg);
    }
    P.d_classes = P.dalloc<ClassDesc>(cls.size());
    P.d_work_off = P.dalloc<uint64_t>(woff.size());
    P.d_tgroups = P.dalloc<GroupDesc>(tg.size());
    P.upload(P.d_classes, cls.data(), cls.size() * sizeof(ClassDesc));
    P.upload(P.d_work_off, woff.data(), woff.size() * sizeof(uint64_t));
    P.upload(P.d_tgroups, tg.data(), tg.size() * sizeof(GroupDesc));
    P.tiled_classes = (int64_t)cls.size();
    P.tiled_work = woff.back();
}

template <int B> unsigned adj_grid(int n)
{
    static unsigned cached = 0;
    if (!cached) {
        int dev = 0, cus = 0, per = 0;
        QF_HIP(hipGetDevice(&dev));
        QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(k_adjoint_block<B, adj_threads(B)>), adj_threads(B), 0));
        cached = (unsigned)std::max(1, std::min(cus * std::max(per, 1), kMaxBlocks));
    }
    return (unsigned)std::min<uint64_t>(cached, 1ull << (n - B));
}

void set_block_bits(qf_plan &P, int B)
{
    if (B != 0 && (B < 6 || B > 12 || B > P.n))
        raise(QF_E_ARG, "blocked apply needs 6 <= block bits <= min(12, n_qubits), or 0");
    void *old[] = {P.d_lruns, P.d_atrip, P.d_alruns, P.d_apairs, P.d_asmap, P.d_apart, P.d_ablocked};
    for (void *p : old)
        P.release(p);
    P.d_lruns = nullptr;
    P.d_atrip = nullptr;
    P.d_asmap = nullptr;
    P.d_alruns = nullptr;
    P.d_apairs = nullptr;
    P.d_apart = nullptr;
    P.d_ablocked = nullptr;
    P.adj_grid = 0;
    P.segs.clear();
    P.asegs.clear();
    P.aseg_k0.clear();
    P.aseg_nstr.clear();
    P.block_bits = B;
    // the adjoint holds two sub-cubes (phi, lambda) in LDS: at most 2^11 each
    P.adj_bits = B >= 10 ? std::min(B, 11) : 0;
    if (!B || P.runs.empty())
        return;
    std::vector<LocalRun> lr;
    build_segments(P.runs, P.n, B, std::min(kApplyQ0, B), P.segs, lr);
    if (B == 12) {
        // triple flags in the flip runs' free itm[1] (the kernel tests them on
        // the descriptor it loads anyway)
        const std::vector<ApplyTriple> at = apply_triples(P.segs, lr);
        for (size_t i = 0; i < lr.size(); i++)
            if (lr[i].x)
                lr[i].itm[1] = at[i].w0 & 3u;
        P.d_atrip = P.dalloc<ApplyTriple>(at.size());
        if (!at.empty())
            P.upload(P.d_atrip, at.data(), at.size() * sizeof(ApplyTriple));
    }
    P.d_lruns = P.dalloc<LocalRun>(lr.size());
    if (!lr.empty())
        P.upload(P.d_lruns, lr.data(), lr.size() * sizeof(LocalRun));
    if (P.adj_bits) {
        // (a pool plan only runs the read-only sweep: longer segments, no tables)
        build_segments(P.runs, P.n, P.adj_bits, kAdjQ0, P.asegs, lr, P.is_pool ? kPoolRuns : kAdjRuns,
                       P.is_pool ? kSegTab : kAdjTab);
        for (const Segment &sg : P.asegs) {
            const int k0 = sg.Q ? lr[(size_t)sg.r0].k0 : 0;
            P.aseg_k0.push_back(k0);
            P.aseg_nstr.push_back(sg.Q ? lr[(size_t)sg.r1 - 1].k0 + lr[(size_t)sg.r1 - 1].m - k0 : 0);
        }
        P.d_alruns = P.dalloc<LocalRun>(lr.size());
        if (!lr.empty())
            P.upload(P.d_alruns, lr.data(), lr.size() * sizeof(LocalRun));
        if (P.adj_bits == 11) {
            const std::vector<AdjPair> ap = adjoint_pairs(P.asegs, lr);
            P.d_apairs = P.dalloc<AdjPair>(ap.size());
            if (!ap.empty())
                P.upload(P.d_apairs, ap.data(), ap.size() * sizeof(AdjPair));
        }
        // string k of local run r: Walsh column e_k (rank <= 3) or k, the sign of s_k
        std::vector<uint32_t> smap((size_t)P.K, 0u);
        for (const Segment &sg : P.asegs) {
            if (!sg.Q)
                continue;
            for (int r = sg.r0; r < sg.r1; r++) {
                const LocalRun &L = lr[(size_t)r];
                const bool walsh = L.r <= 3;
                for (int k = 0; k < L.m; k++)
                    smap[(size_t)(L.k0 + k)] = (uint32_t)(walsh ? L.e[k] : k) | (walsh && L.s[k] < 0 ? 8u : 0u) |
                                               (uint32_t)(r - sg.r0) << 4;
            }
        }
        P.d_asmap = P.dalloc<uint32_t>((size_t)P.K);
        P.upload(P.d_asmap, smap.data(), smap.size() * sizeof(uint32_t));
        std::vector<uint8_t> blocked((size_t)P.K, 0);
        for (size_t i = 0; i < P.asegs.size(); i++)
            for (int t = 0; t < P.aseg_nstr[i]; t++)
                blocked[(size_t)(P.aseg_k0[i] + t)] = 1;
        P.d_ablocked = P.dalloc<uint8_t>((size_t)P.K);
        P.upload(P.d_ablocked, blocked.data(), blocked.size());
        P.adj_grid = P.adj_bits == 10 ? adj_grid<10>(P.n) : adj_grid<11>(P.n);
        P.d_apart = P.dalloc<double>((size_t)P.adj_grid * (size_t)P.K);
    }
}

// Plan tables on the device.  block_bits / energy_tile < 0 take the
// defaults (blocked apply over min(12, n) qubits from 6 qubits up; merged
// energy tiles of 2^11 from 16 qubits up); otherwise as qf_plan_set_block_bits
// and qf_plan_set_energy_tile (merged) would set them.
void plan_init(qf_plan &P, int n, const qf_term *A, int64_t K, const qf_term *H, const int64_t *goff,
               int64_t G, int block_bits = -1, int energy_tile = -1)
{
    if (n < 1 || n > QF_MAX_QUBITS)
        raise(QF_E_RANGE, "n_qubits=" + std::to_string(n) + " out of range [1, " + std::to_string(QF_MAX_QUBITS) + "]");
    if (K < 0 || G < 0)
        raise(QF_E_ARG, "negative term or group count");
    if ((K > 0 && !A) || (G > 0 && (!H || !goff)))
        raise(QF_E_ARG, "null term table");
    if (K > (int64_t)1 << 30 || G > (int64_t)1 << 30)
        raise(QF_E_ARG, "term table too large");
    P.n = n;
    P.K = K;
    if (K > 0) {
        check_terms("ansatz", n, A, K);
        P.runs = make_runs(A, K, P.tab_entries);
        P.ac.resize((size_t)K);
        for (int64_t k = 0; k < K; k++)
            P.ac[(size_t)k] = A[k].c;
        P.d_runs = P.dalloc<RunDesc>(P.runs.size());
        P.d_theta = P.dalloc<double>((size_t)K);
        P.d_tab = P.dalloc<double2>((size_t)P.tab_entries);
        P.d_grad = P.dalloc<double>((size_t)K);
        P.d_pidx = P.dalloc<uint64_t>((size_t)K);
        P.d_pout = P.dalloc<double2>((size_t)K);
        P.upload(P.d_runs, P.runs.data(), P.runs.size() * sizeof(RunDesc));
        set_block_bits(P, block_bits >= 0 ? block_bits : n >= 6 ? std::min(n, 12) : 0);
        // pinned staging for theta (an arena plan stages nothing: freeing
        // pinned memory may wait for the device, which a serving loop avoids)
        if (P.mem == qf_plan::kOwned) {
            QF_HIP(hipHostMalloc((void **)&P.h_theta, (size_t)K * sizeof(double), hipHostMallocDefault));
            QF_HIP(hipEventCreateWithFlags(&P.theta_done, hipEventDisableTiming));
        }
    }
    if (G > 0) {
        std::vector<GroupDesc> gd;
        std::vector<uint32_t> zs;
        std::vector<double> cs;
        build_groups(n, H, goff, G, gd, zs, cs);
        const int64_t KH = goff[G];
        P.G = (int)G;
        P.d_groups = P.dalloc<GroupDesc>((size_t)G);
        P.d_z = P.dalloc<uint32_t>((size_t)KH);
        P.d_c = P.dalloc<double>((size_t)KH);
        P.upload(P.d_groups, gd.data(), gd.size() * sizeof(GroupDesc));
        P.upload(P.d_z, zs.data(), zs.size() * sizeof(uint32_t));
        P.upload(P.d_c, cs.data(), cs.size() * sizeof(double));
        P.groups = gd;
        P.hz = zs;
        P.hc = cs;
        if (n > kSsL && P.sigma_tables) {
            std::vector<SsCls> ssc;
            std::vector<uint32_t> ssw;
            std::vector<SsLo> ssl;
            sigma_stream_tables(gd, zs, cs, kSsNT, ssc, ssw, ssl);
            P.d_ss_cls = P.dalloc<SsCls>(ssc.size());
            P.d_ss_words = P.dalloc<uint32_t>(ssw.size());
            P.d_ss_los = P.dalloc<SsLo>(ssl.size());
            P.upload(P.d_ss_cls, ssc.data(), ssc.size() * sizeof(SsCls));
            P.upload(P.d_ss_words, ssw.data(), ssw.size() * sizeof(uint32_t));
            P.upload(P.d_ss_los, ssl.data(), ssl.size() * sizeof(SsLo));
            P.n_ss_cls = (int)ssc.size();
        }
        for (const GroupDesc &g : gd)
            if (g.k1 > g.kre)
                P.has_imag = true;
        set_energy_tile(P, energy_tile >= 0 ? energy_tile : n >= 16 ? 11 : 0, true);
    }
    P.d_partials = P.dalloc<double>((size_t)kMaxBlocks * kMaxRun);
    P.d_counter = P.dalloc<unsigned>(1);
    P.d_result = P.dalloc<double>(4);
    P.d_dots = P.dalloc<double>(4 * kMaxDots);
    if (P.mem == qf_plan::kOwned) {
        QF_HIP(hipMemset(P.d_counter, 0, sizeof(unsigned)));
    } else if (P.mem == qf_plan::kRegion) {
        // a kernel, not a memset node, so that the clear is also safe to capture
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, P.region_stream, P.d_counter, 1u);
        QF_HIP(hipGetLastError());
    }
}

inline unsigned grid_for(uint64_t work, uint64_t per, unsigned cap)
{
    uint64_t g = (work + per - 1) / per;
    if (g < 1)
        g = 1;
    if (cap && g > cap)
        g = cap;
    return (unsigned)g;
}

void upload_theta(qf_plan &P, const double *theta, hipStream_t s)
{
    if (!theta)
        raise(QF_E_ARG, "theta is NULL");
    if (P.h_theta) {
        QF_HIP(hipEventSynchronize(P.theta_done));  // previous upload has left the staging buffer
        std::memcpy(P.h_theta, theta, (size_t)P.K * sizeof(double));
        QF_HIP(hipMemcpyAsync(P.d_theta, P.h_theta, (size_t)P.K * sizeof(double), hipMemcpyHostToDevice, s));
        QF_HIP(hipEventRecord(P.theta_done, s));
    } else {
        // from the caller's memory, which may be reused once the copy is done
        QF_HIP(hipMemcpyAsync(P.d_theta, theta, (size_t)P.K * sizeof(double), hipMemcpyHostToDevice, s));
        QF_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(k_run_tables, dim3((unsigned)P.runs.size()), dim3(64), 0, s, P.d_runs, P.d_theta,
                       P.d_tab);
    QF_HIP(hipGetLastError());
}

void launch_one_run(qf_plan &P, double2 *psi, const RunDesc &d, double sgn, hipStream_t s)
{
    const uint64_t dim = 1ull << P.n;
    if (d.x) {
        const uint64_t np = dim >> 1;
        hipLaunchKernelGGL(k_apply_run, dim3(grid_for(np, (uint64_t)kBlock * kItems, 0)), dim3(kBlock), 0, s, psi,
                           np, d, P.d_tab, sgn);
    } else {
        hipLaunchKernelGGL(k_apply_diag, dim3(grid_for(dim, kBlock, 8 * kMaxBlocks)), dim3(kBlock), 0, s, psi, dim,
                           d, P.d_tab, sgn);
    }
}

template <int B> void launch_block(qf_plan &P, double2 *psi, const Segment &sg, double sgn, hipStream_t s)
{
    // 512 threads (8 waves) per sub-cube: enough loads in flight per CU at
    // 2^11..2^12 elements while the LDS image still admits two workgroups.
    constexpr int NT = (1 << B) < 512 ? (1 << B) : 512;
    hipLaunchKernelGGL((k_apply_block<B, NT>), dim3((unsigned)(1ull << (P.n - B))), dim3(NT), 0, s, psi, sg,
                       P.d_lruns, P.d_atrip, P.d_tab, sgn);
}

void launch_runs(qf_plan &P, double2 *psi, bool inverse, hipStream_t s)
{
    const uint64_t dim = 1ull << P.n;
    if (P.block_bits) {
        const size_t S = P.segs.size();
        const double sgn = inverse ? -1.0 : 1.0;
        for (size_t i = 0; i < S; i++) {
            const Segment &sg = P.segs[inverse ? S - 1 - i : i];
            if (!sg.Q) {
                launch_one_run(P, psi, P.runs[(size_t)sg.r0], sgn, s);
                continue;
            }
            switch (P.block_bits) {
            case 6: launch_block<6>(P, psi, sg, sgn, s); break;
            case 7: launch_block<7>(P, psi, sg, sgn, s); break;
            case 8: launch_block<8>(P, psi, sg, sgn, s); break;
            case 9: launch_block<9>(P, psi, sg, sgn, s); break;
            case 10: launch_block<10>(P, psi, sg, sgn, s); break;
            case 11: launch_block<11>(P, psi, sg, sgn, s); break;
            default: launch_block<12>(P, psi, sg, sgn, s); break;
            }
        }
        QF_HIP(hipGetLastError());
        return;
    }
    const size_t R = P.runs.size();
    for (size_t i = 0; i < R; i++) {
        const RunDesc &d = P.runs[inverse ? R - 1 - i : i];
        const double sgn = inverse ? -1.0 : 1.0;
        if (d.x) {
            const uint64_t np = dim >> 1;
            hipLaunchKernelGGL(k_apply_run, dim3(grid_for(np, (uint64_t)kBlock * kItems, 0)), dim3(kBlock), 0, s,
                               psi, np, d, P.d_tab, sgn);
        } else {
            hipLaunchKernelGGL(k_apply_diag, dim3(grid_for(dim, kBlock, 8 * kMaxBlocks)), dim3(kBlock), 0, s,
                               psi, dim, d, P.d_tab, sgn);
        }
    }
    QF_HIP(hipGetLastError());
}

void launch_prepare(double2 *psi, int n, uint64_t occ, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    hipLaunchKernelGGL(k_prepare, dim3(grid_for(dim, kBlock, 8 * kMaxBlocks)), dim3(kBlock), 0, s, psi, dim,
                       (uint32_t)occ);
    QF_HIP(hipGetLastError());
}

template <int LT> unsigned tiled_grid(uint64_t work)
{
    static unsigned cached = 0;
    if (!cached) {
        int dev = 0, cus = 0, per = 0;
        QF_HIP(hipGetDevice(&dev));
        QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(k_energy_tiled<LT>), kBlock, 0));
        cached = (unsigned)std::max(1, std::min(cus * std::max(per, 1), kMaxBlocks));
    }
    return (unsigned)std::min<uint64_t>(cached, std::max<uint64_t>(work, 1));
}

constexpr int ni_for(int LT) { return ((1 << LT) / kBlock) >= 8 ? 8 : ((1 << LT) / kBlock); }

template <int LT> unsigned merged_grid(uint64_t work)
{
    static unsigned cached = 0;
    if (!cached) {
        int dev = 0, cus = 0, per = 0;
        QF_HIP(hipGetDevice(&dev));
        QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(k_energy_merged<LT, ni_for(LT)>), kBlock, 0));
        cached = (unsigned)std::max(1, std::min(cus * std::max(per, 1), kMaxBlocks));
    }
    return (unsigned)std::min<uint64_t>(cached, std::max<uint64_t>(work, 1));
}

template <bool IMAG> unsigned stream_grid()
{
    static unsigned cached = 0;
    if (!cached) {
        int dev = 0, cus = 0, per = 0;
        QF_HIP(hipGetDevice(&dev));
        QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(k_energy_stream<IMAG>), kBlock, 0));
        cached = (unsigned)std::max(1, std::min(cus * std::max(per, 1), kMaxBlocks));
    }
    return cached;
}

template <int LT> void launch_energy_tiled(qf_plan &P, const double2 *psi, double *dev_out, hipStream_t s)
{
    if (P.merged && LT == 11 && P.d_vcls) {
        if (P.has_imag)
            hipLaunchKernelGGL(k_energy_stream<true>, dim3(stream_grid<true>()), dim3(kBlock), 0, s, psi, P.d_vcls,
                               P.n_vcls, P.per_vcls, P.d_tgroups, P.d_recs, P.d_partials, P.d_counter, dev_out);
        else
            hipLaunchKernelGGL(k_energy_stream<false>, dim3(stream_grid<false>()), dim3(kBlock), 0, s, psi,
                               P.d_vcls, P.n_vcls, P.per_vcls, P.d_tgroups, P.d_recs, P.d_partials, P.d_counter,
                               dev_out);
        QF_HIP(hipGetLastError());
        return;
    }
    if (P.merged) {
        hipLaunchKernelGGL((k_energy_merged<LT, ni_for(LT)>), dim3(merged_grid<LT>(P.tiled_work)), dim3(kBlock), 0, s,
                           psi, P.d_classes, P.d_work_off, P.tiled_work, P.d_tgroups, P.d_recs,
                           P.d_partials, P.d_counter, dev_out);
        QF_HIP(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL(k_energy_tiled<LT>, dim3(tiled_grid<LT>(P.tiled_work)), dim3(kBlock), 0, s, psi,
                       P.d_classes, P.d_work_off, P.tiled_work, P.d_tgroups, P.d_z, P.d_c, P.d_partials,
                       P.d_counter, dev_out);
    QF_HIP(hipGetLastError());
}

void launch_energy(qf_plan &P, const double2 *psi, double *dev_out, hipStream_t s)
{
    switch (P.tile_bits) {
    case 10:
        return launch_energy_tiled<10>(P, psi, dev_out, s);
    case 11:
        return launch_energy_tiled<11>(P, psi, dev_out, s);
    case 12:
        return launch_energy_tiled<12>(P, psi, dev_out, s);
    default:
        break;
    }
    const uint64_t np = 1ull << (P.n - 1 > 0 ? P.n - 1 : 0);
    const unsigned nb = grid_for(np, (uint64_t)kBlock * kItems, kMaxBlocks);
    hipLaunchKernelGGL(k_energy, dim3(nb), dim3(kBlock), 0, s, psi, P.n, P.d_groups, P.G, P.d_z, P.d_c,
                       P.d_partials, P.d_counter, dev_out);
    QF_HIP(hipGetLastError());
}

template <bool IMAG> unsigned sigma_stream_grid()
{
    static unsigned cached = 0;
    if (!cached) {
        int dev = 0, cus = 0, per = 0;
        QF_HIP(hipGetDevice(&dev));
        QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(k_sigma_stream<IMAG>), kSsNT, 0));
        cached = (unsigned)std::max(1, std::min(cus * std::max(per, 1), kMaxBlocks));
    }
    return cached;
}

void launch_sigma(qf_plan &P, const double2 *psi, double2 *lam, double *dev_out, hipStream_t s)
{
    if (P.n_ss_cls) {
        const unsigned ntiles = 1u << (P.n - kSsL);
        if (P.has_imag)
            hipLaunchKernelGGL(k_sigma_stream<true>, dim3(std::min(ntiles, sigma_stream_grid<true>())),
                               dim3(kSsNT), 0, s, psi, lam, P.n, P.d_ss_cls, P.n_ss_cls, P.d_ss_words,
                               P.d_ss_los, P.d_partials, P.d_counter, dev_out);
        else
            hipLaunchKernelGGL(k_sigma_stream<false>, dim3(std::min(ntiles, sigma_stream_grid<false>())),
                               dim3(kSsNT), 0, s, psi, lam, P.n, P.d_ss_cls, P.n_ss_cls, P.d_ss_words,
                               P.d_ss_los, P.d_partials, P.d_counter, dev_out);
        QF_HIP(hipGetLastError());
        return;
    }
    const uint64_t dim = 1ull << P.n;
    const unsigned nb = grid_for(dim, (uint64_t)kBlock * kItems, kMaxBlocks);
    hipLaunchKernelGGL(k_sigma, dim3(nb), dim3(kBlock), 0, s, psi, lam, P.n, P.d_groups, P.G, P.d_z, P.d_c,
                       P.d_partials, P.d_counter, dev_out);
    QF_HIP(hipGetLastError());
}

void launch_adjoint_run(qf_plan &P, double2 *phi, double2 *lam, const RunDesc &d, hipStream_t s)
{
    const uint64_t np = d.x ? (1ull << P.n) >> 1 : 1ull << P.n;
    hipLaunchKernelGGL(k_adjoint_run, dim3(grid_for(np, (uint64_t)kBlock * kItems, kMaxBlocks)), dim3(kBlock), 0, s,
                       phi, lam, np, d, P.d_tab, P.d_partials, P.d_counter, P.d_grad);
}


void launch_adjoint(qf_plan &P, double2 *phi, double2 *lam, hipStream_t s)
{
    if (P.is_pool)  // its segments exceed the undoing sweep's kAdjRuns
        raise(QF_E_ARG, "reverse sweep: a pool plan only takes the read-only sweep");
    if (P.adj_bits) {
        for (size_t i = P.asegs.size(); i-- > 0;) {
            const Segment &sg = P.asegs[i];
            if (!sg.Q) {
                launch_adjoint_run(P, phi, lam, P.runs[(size_t)sg.r0], s);
                continue;
            }
            const int sk0 = P.aseg_k0[i], nstr = P.aseg_nstr[i];
            if (P.adj_bits == 10)
                hipLaunchKernelGGL((k_adjoint_block<10, adj_threads(10)>), dim3(P.adj_grid), dim3(adj_threads(10)),
                                   0, s, phi, lam, P.n, sg, P.d_alruns, P.d_apairs, P.d_asmap, P.d_tab, sk0, nstr, P.d_apart,
                                   (int)P.K);
            else
                hipLaunchKernelGGL((k_adjoint_block<11, adj_threads(11)>), dim3(P.adj_grid), dim3(adj_threads(11)),
                                   0, s, phi, lam, P.n, sg, P.d_alruns, P.d_apairs, P.d_asmap, P.d_tab, sk0, nstr, P.d_apart,
                                   (int)P.K);
        }
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((P.K + 63) / 64)), dim3(kBlock), 0, s, P.d_apart,
                           (int)P.adj_grid, (int)P.K, P.d_ablocked, P.d_grad);
        QF_HIP(hipGetLastError());
        return;
    }
    for (size_t i = P.runs.size(); i-- > 0;)
        launch_adjoint_run(P, phi, lam, P.runs[i], s);
    QF_HIP(hipGetLastError());
}

// String sums 2 Im <lambda|P_k|phi> of every string of a pool plan, with phi
// and lambda left unchanged: the blocked sweep's segments read-only, runs
// too wide for a sub-cube through the one-run kernel with identity tables.
void launch_pool_sweep(qf_plan &Q, double2 *phi, double2 *lam, hipStream_t s)
{
    if (Q.adj_bits) {
        for (size_t i = 0; i < Q.asegs.size(); i++) {
            const Segment &sg = Q.asegs[i];
            if (!sg.Q) {
                launch_adjoint_run(Q, phi, lam, Q.runs[(size_t)sg.r0], s);
                continue;
            }
            const int sk0 = Q.aseg_k0[i], nstr = Q.aseg_nstr[i];
            if (Q.adj_bits == 10)
                hipLaunchKernelGGL((k_adjoint_block<10, adj_threads(10), false>), dim3(Q.adj_grid),
                                   dim3(adj_threads(10)), 0, s, phi, lam, Q.n, sg, Q.d_alruns, nullptr, Q.d_asmap, Q.d_tab,
                                   sk0, nstr, Q.d_apart, (int)Q.K);
            else
                hipLaunchKernelGGL((k_adjoint_block<11, adj_threads(11), false>), dim3(Q.adj_grid),
                                   dim3(adj_threads(11)), 0, s, phi, lam, Q.n, sg, Q.d_alruns, nullptr, Q.d_asmap, Q.d_tab,
                                   sk0, nstr, Q.d_apart, (int)Q.K);
        }
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((Q.K + 63) / 64)), dim3(kBlock), 0, s, Q.d_apart,
                           (int)Q.adj_grid, (int)Q.K, Q.d_ablocked, Q.d_grad);
        QF_HIP(hipGetLastError());
        return;
    }
    for (size_t i = 0; i < Q.runs.size(); i++)
        launch_adjoint_run(Q, phi, lam, Q.runs[i], s);
    QF_HIP(hipGetLastError());
}

void fetch(double *host, const double *dev, size_t count, hipStream_t s)
{
    QF_HIP(hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipStreamSynchronize(s));
}

void need_ansatz(const qf_plan *P)
{
    if (!P)
        raise(QF_E_ARG, "plan is NULL");
}

void energy_grad_impl(qf_plan &P, uint64_t occ, const double *theta, void *workspace, double *E_out,
                      double *grad, hipStream_t s)
{
    if (!workspace || !E_out || (P.K > 0 && !grad))
        raise(QF_E_ARG, "energy_grad: null workspace or output");
    if (P.G == 0)
        raise(QF_E_ARG, "energy_grad: plan has no Hamiltonian");
    if (occ >> P.n)
        raise(QF_E_RANGE, "occ_mask has a bit >= n_qubits");
    double2 *phi = (double2 *)workspace;
    double2 *lam = phi + (1ull << P.n);
    launch_prepare(phi, P.n, occ, s);
    if (P.K > 0) {
        upload_theta(P, theta, s);
        launch_runs(P, phi, false, s);
    }
    launch_sigma(P, phi, lam, P.d_result, s);
    if (P.K > 0)
        launch_adjoint(P, phi, lam, s);
    QF_HIP(hipMemcpyAsync(E_out, P.d_result, sizeof(double), hipMemcpyDeviceToHost, s));
    if (P.K > 0)
        QF_HIP(hipMemcpyAsync(grad, P.d_grad, (size_t)P.K * sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipStreamSynchronize(s));
}

// A pool plan: members sorted by the flip mask of their strings (stable), the
// strings concatenated in that order as the plan's ansatz, identity (cos,
// sin) tables for the runs that go through the one-run kernel.
void pool_init(qf_plan &Q, int n, const qf_term *pool, const int64_t *pool_off, int64_t n_pool)
{
    if (n_pool < 1 || !pool || !pool_off)
        raise(QF_E_ARG, "pool: needs at least one member");
    if (pool_off[0] != 0)
        raise(QF_E_ARG, "pool: pool_off[0] must be 0");
    for (int64_t i = 0; i < n_pool; i++) {
        if (pool_off[i + 1] <= pool_off[i])
            raise(QF_E_ARG, "pool: member " + std::to_string(i) + " has no strings");
        for (int64_t k = pool_off[i] + 1; k < pool_off[i + 1]; k++)
            if (pool[k].x != pool[pool_off[i]].x)
                raise(QF_E_ARG, "pool: the strings of member " + std::to_string(i) + " differ in flip mask");
    }
    std::vector<int64_t> order((size_t)n_pool);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return pool[pool_off[a]].x < pool[pool_off[b]].x; });
    std::vector<qf_term> sorted;
    sorted.reserve((size_t)pool_off[n_pool]);
    Q.pool_off.assign(1, 0);
    for (int64_t i : order) {
        for (int64_t k = pool_off[i]; k < pool_off[i + 1]; k++)
            sorted.push_back(pool[k]);
        Q.pool_off.push_back((int64_t)sorted.size());
    }
    Q.pool_perm = order;
    Q.pool_c.resize(sorted.size());
    for (size_t k = 0; k < sorted.size(); k++)
        Q.pool_c[k] = sorted[k].c;
    Q.is_pool = true;  // before the segments are built (longer read-only segments)
    plan_init(Q, n, sorted.data(), (int64_t)sorted.size(), nullptr, nullptr, 0);
    std::vector<double> zero(sorted.size(), 0.0);
    upload_theta(Q, zero.data(), nullptr);
    QF_HIP(hipStreamSynchronize(nullptr));
}

// E and g_nu = -sum_k c_k (2 Im <lambda|P_k|psi>) for Psi = U(theta) Phi.
void pool_grad_impl(qf_plan &P, qf_plan &Q, uint64_t occ, const double *theta, void *workspace, double *E_out,
                    double *g_out, hipStream_t s)
{
    if (!Q.is_pool)
        raise(QF_E_ARG, "pool_grad: the second plan is not a pool plan");
    if (Q.n != P.n)
        raise(QF_E_ARG, "pool_grad: plan and pool have different qubit counts");
    if (!workspace || !E_out || !g_out)
        raise(QF_E_ARG, "pool_grad: null workspace or output");
    if (P.G == 0)
        raise(QF_E_ARG, "pool_grad: plan has no Hamiltonian");
    if (occ >> P.n)
        raise(QF_E_RANGE, "occ_mask has a bit >= n_qubits");
    double2 *phi = (double2 *)workspace;
    double2 *lam = phi + (1ull << P.n);
    launch_prepare(phi, P.n, occ, s);
    if (P.K > 0) {
        upload_theta(P, theta, s);
        launch_runs(P, phi, false, s);
    }
    launch_sigma(P, phi, lam, P.d_result, s);
    launch_pool_sweep(Q, phi, lam, s);
    std::vector<double> gk((size_t)Q.K);
    QF_HIP(hipMemcpyAsync(E_out, P.d_result, sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipMemcpyAsync(gk.data(), Q.d_grad, (size_t)Q.K * sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i + 1 < Q.pool_off.size(); i++) {
        double v = 0.0;
        for (int64_t k = Q.pool_off[i]; k < Q.pool_off[i + 1]; k++)
            v += -Q.pool_c[(size_t)k] * gk[(size_t)k];
        g_out[Q.pool_perm[i]] = v;
    }
}

// PQE residuals (Sec. 3.3): r_mu = s_mu [U^dagger H U Phi_0](d_mu): the
// forward pass, lambda = H psi, lambda <- U^dagger lambda (the runs undone in
// reverse), then the amplitudes of lambda at the excited determinants.
void pqe_impl(qf_plan &P, uint64_t occ, const double *theta, const uint64_t *det, const int *sign, int64_t n_res,
              void *workspace, double *E_out, double *r_out, hipStream_t s)
{
    if (!workspace || !E_out || (n_res > 0 && (!det || !sign || !r_out)))
        raise(QF_E_ARG, "pqe_residuals: null workspace, determinants or output");
    if (P.G == 0 || P.K == 0)
        raise(QF_E_ARG, "pqe_residuals: the plan needs an ansatz and a Hamiltonian");
    if (n_res < 0 || n_res > P.K)
        raise(QF_E_ARG, "pqe_residuals: between 0 and K residuals");
    if (occ >> P.n)
        raise(QF_E_RANGE, "occ_mask has a bit >= n_qubits");
    for (int64_t i = 0; i < n_res; i++)
        if (det[i] >> P.n)
            raise(QF_E_RANGE, "pqe_residuals: determinant " + std::to_string(i) + " has a bit >= n_qubits");
    double2 *phi = (double2 *)workspace;
    double2 *lam = phi + (1ull << P.n);
    launch_prepare(phi, P.n, occ, s);
    upload_theta(P, theta, s);
    launch_runs(P, phi, false, s);
    launch_sigma(P, phi, lam, P.d_result, s);
    launch_runs(P, lam, true, s);
    std::vector<double2> amp((size_t)std::max<int64_t>(n_res, 1));
    if (n_res > 0) {
        QF_HIP(hipMemcpyAsync(P.d_pidx, det, (size_t)n_res * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather, dim3(grid_for((uint64_t)n_res, kBlock, 64)), dim3(kBlock), 0, s, lam, P.d_pidx,
                           n_res, P.d_pout);
        QF_HIP(hipGetLastError());
        QF_HIP(hipMemcpyAsync(amp.data(), P.d_pout, (size_t)n_res * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    QF_HIP(hipMemcpyAsync(E_out, P.d_result, sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n_res; i++)
        r_out[i] = (double)sign[i] * amp[(size_t)i].x;
}

// psi <- (prod_k exp(-i t c_k P_k / r))^r psi over the plan's ansatz strings
// (Sec. 3.7, Eq. (m_trotter_step2) with the Hamiltonian's strings as the
// ansatz): theta_k = t c_k / r, the fused runs applied r times.
void trotter_impl(qf_plan &P, double2 *psi, double t, int r, hipStream_t s)
{
    if (P.K == 0)
        raise(QF_E_ARG, "trotter: the plan has no strings to exponentiate");
    if (r < 1)
        raise(QF_E_ARG, "trotter: r must be >= 1");
    std::vector<double> th((size_t)P.K);
    for (int64_t k = 0; k < P.K; k++)
        th[(size_t)k] = t * P.ac[(size_t)k] / (double)r;
    upload_theta(P, th.data(), s);
    for (int i = 0; i < r; i++)
        launch_runs(P, psi, false, s);
}

void dots(qf_plan &P, const double2 *a, const double2 *b, const double2 *xs, int J, hipStream_t s)
{
    const uint64_t dim = 1ull << P.n;
    // partials hold kMaxBlocks * kMaxRun doubles: 4 * JMAX per block
    if (J <= 4) {
        const unsigned nb = grid_for(dim, (uint64_t)kBlock * 4, (unsigned)(kMaxBlocks * kMaxRun / 16));
        hipLaunchKernelGGL(k_dots<4>, dim3(nb), dim3(kBlock), 0, s, a, b, xs, dim, J, P.d_partials, P.d_counter,
                           P.d_dots);
    } else {
        const unsigned nb = grid_for(dim, (uint64_t)kBlock * 4, (unsigned)(kMaxBlocks * kMaxRun / 64));
        hipLaunchKernelGGL(k_dots<kMaxDots>, dim3(nb), dim3(kBlock), 0, s, a, b, xs, dim, J, P.d_partials,
                           P.d_counter, P.d_dots);
    }
    QF_HIP(hipGetLastError());
}

// QK basis psi_k = Trotter(k dt, r) |occ>, k = 0 .. s, in states[0 .. s];
// states[s + 1] holds H psi_m in turn.  S[m][k] = <psi_m|psi_k>,
// Hm[m][k] = <H psi_m|psi_k> = <psi_m|H|psi_k>, complex, row-major.
void qk_impl(qf_plan &P, uint64_t occ, double dt, int s_max, int r, double2 *states, double *S, double *Hm,
             hipStream_t s)
{
    if (P.G == 0 || P.K == 0)
        raise(QF_E_ARG, "qk_matrices: the plan needs the Hamiltonian as both ansatz and Hamiltonian");
    if (s_max < 0 || s_max + 1 > kMaxDots)
        raise(QF_E_ARG, "qk_matrices: 0 <= s < " + std::to_string(kMaxDots));
    if (!states || !S || !Hm)
        raise(QF_E_ARG, "qk_matrices: null states or output");
    if (occ >> P.n)
        raise(QF_E_RANGE, "occ_mask has a bit >= n_qubits");
    const uint64_t dim = 1ull << P.n;
    const int J = s_max + 1;
    for (int k = 0; k < J; k++) {
        launch_prepare(states + (uint64_t)k * dim, P.n, occ, s);
        if (k > 0)
            trotter_impl(P, states + (uint64_t)k * dim, k * dt, r, s);
    }
    double2 *sig = states + (uint64_t)J * dim;
    const int JM = J <= 4 ? 4 : kMaxDots;
    std::vector<double> out((size_t)4 * JM);
    for (int m = 0; m < J; m++) {
        launch_sigma(P, states + (uint64_t)m * dim, sig, P.d_result, s);
        dots(P, states + (uint64_t)m * dim, sig, states, J, s);
        QF_HIP(hipMemcpyAsync(out.data(), P.d_dots, out.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        QF_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < J; k++) {
            S[2 * (m * J + k)] = out[(size_t)(2 * k)];
            S[2 * (m * J + k) + 1] = out[(size_t)(2 * k + 1)];
            Hm[2 * (m * J + k)] = out[(size_t)(2 * JM + 2 * k)];
            Hm[2 * (m * J + k) + 1] = out[(size_t)(2 * JM + 2 * k + 1)];
        }
    }
}

} // namespace qf

using namespace qf;

extern "C" int qf_plan_trotter(qf_plan *plan, void *psi, double t, int r, void *stream)
{
    return guarded([&]() -> int {
        if (!plan || !psi)
            return fail(QF_E_ARG, "qf_plan_trotter: null plan or state");
        trotter_impl(*plan, (double2 *)psi, t, r, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_plan_qk_matrices(qf_plan *plan, uint64_t occ_mask, double dt, int s, int r, void *states,
                                   double *S_out, double *H_out, void *stream)
{
    return guarded([&]() -> int {
        if (!plan)
            return fail(QF_E_ARG, "qf_plan_qk_matrices: plan is NULL");
        qk_impl(*plan, occ_mask, dt, s, r, (double2 *)states, S_out, H_out, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_plan_pqe_residuals(qf_plan *plan, uint64_t occ_mask, const double *theta, const uint64_t *det,
                                     const int *sign, int64_t n_res, void *workspace, double *E_out, double *r_out,
                                     void *stream)
{
    return guarded([&]() -> int {
        if (!plan)
            return fail(QF_E_ARG, "qf_plan_pqe_residuals: plan is NULL");
        pqe_impl(*plan, occ_mask, theta, det, sign, n_res, workspace, E_out, r_out, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_pqe_residuals(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta, int64_t K,
                                const qf_term *H, const int64_t *group_off, int64_t n_groups, const uint64_t *det,
                                const int *sign, int64_t n_res, void *workspace, double *E_out, double *r_out,
                                void *stream)
{
    return guarded([&]() -> int {
        if (n_groups < 1 || K < 1)
            return fail(QF_E_ARG, "qf_pqe_residuals: needs an ansatz and a Hamiltonian");
        qf_plan P;
        plan_init(P, n_qubits, A, K, H, group_off, n_groups);
        pqe_impl(P, occ_mask, theta, det, sign, n_res, workspace, E_out, r_out, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_plan_pqe_solve(qf_plan *plan, uint64_t occ_mask, const qf_term *A, const int64_t *exc_off,
                                 int64_t n_par, const uint64_t *det, const int *sign, const double *delta,
                                 double *t, int max_iter, double tol, void *workspace, double *E_out, double *r_out,
                                 int *iters, void *stream)
{
    return guarded([&]() -> int {
        if (!plan || !A || !exc_off || !det || !sign || !delta || !t || !r_out || !iters || max_iter < 0)
            return fail(QF_E_ARG, "qf_plan_pqe_solve: bad arguments");
        if (n_par < 1 || exc_off[n_par] != plan->K)
            return fail(QF_E_ARG, "qf_plan_pqe_solve: exc_off does not cover the plan's ansatz");
        for (int64_t mu = 0; mu < n_par; mu++)
            if (delta[mu] == 0.0)
                return fail(QF_E_ARG, "qf_plan_pqe_solve: Delta_%lld is zero", (long long)mu);
        std::vector<double> theta((size_t)plan->K);
        hipStream_t s = (hipStream_t)stream;
        *iters = 0;
        for (int it = 0;; it++) {
            // theta_k = -c_k t_mu (Sec. 3.1 product of exponentials)
            for (int64_t mu = 0; mu < n_par; mu++)
                for (int64_t k = exc_off[mu]; k < exc_off[mu + 1]; k++)
                    theta[(size_t)k] = -A[k].c * t[mu];
            pqe_impl(*plan, occ_mask, theta.data(), det, sign, n_par, workspace, E_out, r_out, s);
            double rmax = 0.0;
            for (int64_t mu = 0; mu < n_par; mu++)
                rmax = std::max(rmax, std::fabs(r_out[mu]));
            *iters = it;
            if (rmax < tol || it >= max_iter)
                break;
            // Eq. (fixed_point): t_mu <- t_mu + r_mu / Delta_mu
            for (int64_t mu = 0; mu < n_par; mu++)
                t[mu] += r_out[mu] / delta[mu];
        }
        return QF_OK;
    });
}

extern "C" int qf_plan_create_pool(int n_qubits, const qf_term *pool, const int64_t *pool_off, int64_t n_pool,
                                   qf_plan **out)
{
    return guarded([&]() -> int {
        if (!out)
            return fail(QF_E_ARG, "qf_plan_create_pool: out is NULL");
        *out = nullptr;
        qf_plan *Q = new qf_plan();
        try {
            pool_init(*Q, n_qubits, pool, pool_off, n_pool);
        } catch (...) {
            delete Q;
            throw;
        }
        *out = Q;
        return QF_OK;
    });
}

extern "C" int qf_plan_pool_grad(qf_plan *plan, qf_plan *pool, uint64_t occ_mask, const double *theta,
                                 void *workspace, double *E_out, double *g_out, void *stream)
{
    return guarded([&]() -> int {
        if (!plan || !pool)
            return fail(QF_E_ARG, "qf_plan_pool_grad: null plan");
        pool_grad_impl(*plan, *pool, occ_mask, theta, workspace, E_out, g_out, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_pool_grad(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta, int64_t K,
                            const qf_term *H, const int64_t *group_off, int64_t n_groups, const qf_term *pool,
                            const int64_t *pool_off, int64_t n_pool, void *workspace, double *E_out,
                            double *g_out, void *stream)
{
    return guarded([&]() -> int {
        if (n_groups < 1)
            return fail(QF_E_ARG, "qf_pool_grad: needs a Hamiltonian (n_groups >= 1)");
        qf_plan P, Q;
        plan_init(P, n_qubits, A, K, H, group_off, n_groups);
        pool_init(Q, n_qubits, pool, pool_off, n_pool);
        pool_grad_impl(P, Q, occ_mask, theta, workspace, E_out, g_out, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_plan_create(int n_qubits, const qf_term *A, int64_t K, const qf_term *H,
                              const int64_t *group_off, int64_t n_groups, qf_plan **out)
{
    return guarded([&]() -> int {
        if (!out)
            return fail(QF_E_ARG, "qf_plan_create: out is NULL");
        *out = nullptr;
        qf_plan *P = new qf_plan();
        try {
            plan_init(*P, n_qubits, A, K, H, group_off, n_groups);
        } catch (...) {
            delete P;
            throw;
        }
        *out = P;
        return QF_OK;
    });
}

extern "C" int qf_plan_create_arena(int n_qubits, const qf_term *A, int64_t K, const qf_term *H,
                                    const int64_t *group_off, int64_t n_groups, int block_bits, int energy_tile,
                                    void *arena, int64_t arena_bytes, int64_t *need_bytes, void *stream,
                                    qf_plan **out)
{
    return guarded([&]() -> int {
        if (!need_bytes)
            return fail(QF_E_ARG, "qf_plan_create_arena: need_bytes is NULL");
        if (arena && !out)
            return fail(QF_E_ARG, "qf_plan_create_arena: out is NULL");
        if (out)
            *out = nullptr;
        {
            qf_plan M;
            M.mem = qf_plan::kMeasure;
            plan_init(M, n_qubits, A, K, H, group_off, n_groups, block_bits, energy_tile);
            *need_bytes = (int64_t)M.region_used;
        }
        if (!arena)
            return QF_OK;
        if (reinterpret_cast<uintptr_t>(arena) % 256)
            return fail(QF_E_ARG, "qf_plan_create_arena: arena is not 256-byte aligned");
        if (arena_bytes < *need_bytes)
            return fail(QF_E_SIZE, "qf_plan_create_arena: arena of %lld bytes, plan needs %lld",
                        (long long)arena_bytes, (long long)*need_bytes);
        qf_plan *P = new qf_plan();
        P->mem = qf_plan::kRegion;
        P->region = (char *)arena;
        P->region_cap = (size_t)arena_bytes;
        P->region_stream = (hipStream_t)stream;
        try {
            plan_init(*P, n_qubits, A, K, H, group_off, n_groups, block_bits, energy_tile);
        } catch (...) {
            delete P;
            throw;
        }
        *out = P;
        return QF_OK;
    });
}

extern "C" int qf_plan_destroy(qf_plan *plan)
{
    delete plan;
    return QF_OK;
}

extern "C" int qf_plan_apply(qf_plan *P, void *psi, const double *theta, int inverse, void *stream)
{
    return guarded([&]() -> int {
        if (!P || !psi)
            return fail(QF_E_ARG, "qf_plan_apply: null plan or state");
        if (P->K == 0)
            return QF_OK;
        hipStream_t s = (hipStream_t)stream;
        upload_theta(*P, theta, s);
        launch_runs(*P, (double2 *)psi, inverse != 0, s);
        return QF_OK;
    });
}

extern "C" int qf_plan_energy(qf_plan *P, const void *psi, double *E_out, void *stream)
{
    return guarded([&]() -> int {
        if (!P || !psi || !E_out)
            return fail(QF_E_ARG, "qf_plan_energy: null argument");
        if (P->G == 0) {
            *E_out = 0.0;
            return QF_OK;
        }
        hipStream_t s = (hipStream_t)stream;
        launch_energy(*P, (const double2 *)psi, P->d_result, s);
        fetch(E_out, P->d_result, 1, s);
        return QF_OK;
    });
}

extern "C" int qf_plan_sigma(qf_plan *P, const void *psi, void *lambda, double *E_out, void *stream)
{
    return guarded([&]() -> int {
        if (!P || !psi || !lambda || !E_out)
            return fail(QF_E_ARG, "qf_plan_sigma: null argument");
        if (P->G == 0)
            return fail(QF_E_ARG, "qf_plan_sigma: plan has no Hamiltonian");
        hipStream_t s = (hipStream_t)stream;
        launch_sigma(*P, (const double2 *)psi, (double2 *)lambda, P->d_result, s);
        fetch(E_out, P->d_result, 1, s);
        return QF_OK;
    });
}

extern "C" int qf_plan_energy_grad(qf_plan *P, uint64_t occ_mask, const double *theta, void *workspace,
                                   double *E_out, double *dE_dtheta, void *stream)
{
    return guarded([&]() -> int {
        if (!P)
            return fail(QF_E_ARG, "qf_plan_energy_grad: plan is NULL");
        energy_grad_impl(*P, occ_mask, theta, workspace, E_out, dE_dtheta, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_prepare_state(void *psi, int n_qubits, uint64_t occ_mask, void *stream)
{
    return guarded([&]() -> int {
        if (!psi)
            return fail(QF_E_ARG, "qf_prepare_state: psi is NULL");
        if (n_qubits < 1 || n_qubits > QF_MAX_QUBITS)
            return fail(QF_E_RANGE, "qf_prepare_state: n_qubits=%d out of range [1, %d]", n_qubits, QF_MAX_QUBITS);
        if (occ_mask >> n_qubits)
            return fail(QF_E_RANGE, "qf_prepare_state: occ_mask has a bit >= n_qubits");
        launch_prepare((double2 *)psi, n_qubits, occ_mask, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_apply_pauli_exp(void *psi, int n_qubits, const qf_term *terms, const double *theta,
                                  int64_t K, int inverse, void *stream)
{
    return guarded([&]() -> int {
        if (!psi)
            return fail(QF_E_ARG, "qf_apply_pauli_exp: psi is NULL");
        if (K < 0)
            return fail(QF_E_ARG, "qf_apply_pauli_exp: K < 0");
        if (n_qubits < 1 || n_qubits > QF_MAX_QUBITS)
            return fail(QF_E_RANGE, "qf_apply_pauli_exp: n_qubits=%d out of range", n_qubits);
        if (K == 0)
            return QF_OK;
        if (!terms || !theta)
            return fail(QF_E_ARG, "qf_apply_pauli_exp: null terms or theta");
        qf_plan P;
        plan_init(P, n_qubits, terms, K, nullptr, nullptr, 0);
        hipStream_t s = (hipStream_t)stream;
        upload_theta(P, theta, s);
        launch_runs(P, (double2 *)psi, inverse != 0, s);
        QF_HIP(hipStreamSynchronize(s));  // the temporary plan's buffers are freed on return
        return QF_OK;
    });
}

extern "C" int qf_energy(const void *psi, int n_qubits, const qf_term *H, const int64_t *group_off,
                         int64_t n_groups, double *E_out, void *stream)
{
    return guarded([&]() -> int {
        if (!psi || !E_out)
            return fail(QF_E_ARG, "qf_energy: null psi or E_out");
        if (n_groups < 0)
            return fail(QF_E_ARG, "qf_energy: n_groups < 0");
        if (n_qubits < 1 || n_qubits > QF_MAX_QUBITS)
            return fail(QF_E_RANGE, "qf_energy: n_qubits=%d out of range", n_qubits);
        if (n_groups == 0) {
            *E_out = 0.0;
            return QF_OK;
        }
        qf_plan P;
        plan_init(P, n_qubits, nullptr, 0, H, group_off, n_groups);
        hipStream_t s = (hipStream_t)stream;
        launch_energy(P, (const double2 *)psi, P.d_result, s);
        fetch(E_out, P.d_result, 1, s);
        return QF_OK;
    });
}

namespace qf {
namespace {

// Device memory of qf_energy_static: every table and scratch array of its
// one-shot plan is carved from this array, so the call allocates nothing.
// Each GPU holds its own copy until the process ends; host code must use the
// per-device address from hipGetSymbolAddress, never the array's name.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex scratch_mu;
void *scratch_dev[256];  // per device index

void *scratch_address()
{
    int dev = 0;
    QF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256)
        raise(QF_E_HIP, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            raise(QF_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        scratch_dev[dev] = ptr;
    }
    return scratch_dev[dev];
}

} // namespace
} // namespace qf

extern "C" int qf_energy_static(const void *psi, int n_qubits, const qf_term *H, const int64_t *group_off,
                                int64_t n_groups, double *E_out, void *stream)
{
    return guarded([&]() -> int {
        if (!psi || !E_out)
            return fail(QF_E_ARG, "qf_energy_static: null psi or E_out");
        if (n_groups < 0)
            return fail(QF_E_ARG, "qf_energy_static: n_groups < 0");
        if (n_qubits < 1 || n_qubits > QF_MAX_QUBITS)
            return fail(QF_E_RANGE, "qf_energy_static: n_qubits=%d out of range", n_qubits);
        if (n_groups == 0) {
            *E_out = 0.0;
            return QF_OK;
        }
        hipStream_t s = (hipStream_t)stream;
        qf_plan P;
        P.mem = qf_plan::kRegion;
        P.region = (char *)scratch_address();
        P.region_cap = kStaticScratchBytes;
        P.region_stream = s;
        P.sigma_tables = false;  // energy only
        try {
            plan_init(P, n_qubits, nullptr, 0, H, group_off, n_groups);
        } catch (const Error &e) {
            if (e.status == QF_E_SIZE)
                return fail(QF_E_SIZE, "qf_energy_static: the Hamiltonian's device tables exceed the %zu-byte "
                                       "static scratch", kStaticScratchBytes);
            throw;
        }
        launch_energy(P, (const double2 *)psi, P.d_result, s);
        fetch(E_out, P.d_result, 1, s);
        return QF_OK;
    });
}

extern "C" int qf_energy_grad(int n_qubits, uint64_t occ_mask, const qf_term *A, const double *theta,
                              int64_t K, const qf_term *H, const int64_t *group_off, int64_t n_groups,
                              void *workspace, double *E_out, double *dE_dtheta, void *stream)
{
    return guarded([&]() -> int {
        if (n_groups < 1)
            return fail(QF_E_ARG, "qf_energy_grad: needs a Hamiltonian (n_groups >= 1)");
        qf_plan P;
        plan_init(P, n_qubits, A, K, H, group_off, n_groups);
        energy_grad_impl(P, occ_mask, theta, workspace, E_out, dE_dtheta, (hipStream_t)stream);
        return QF_OK;
    });
}

extern "C" int qf_plan_set_energy_tile(qf_plan *P, int tile_bits, int merged)
{
    return guarded([&]() -> int {
        if (!P)
            return fail(QF_E_ARG, "qf_plan_set_energy_tile: plan is NULL");
        if (P->mem != qf_plan::kOwned)
            return fail(QF_E_ARG, "qf_plan_set_energy_tile: an arena plan fixes its tiles at creation");
        set_energy_tile(*P, tile_bits, merged != 0);
        return QF_OK;
    });
}

extern "C" int qf_plan_info(const qf_plan *P, int *tile_bits, int64_t *classes, int64_t *energy_passes)
{
    if (!P)
        return fail(QF_E_ARG, "qf_plan_info: plan is NULL");
    if (tile_bits)
        *tile_bits = P->merged ? -P->tile_bits : P->tile_bits;
    if (classes)
        *classes = P->tiled_classes;
    if (energy_passes)
        *energy_passes = P->tile_bits ? P->tiled_classes : P->G;
    return QF_OK;
}

extern "C" int qf_plan_grad_info(const qf_plan *P, int64_t *sigma_passes, int64_t *sweep_passes)
{
    if (!P)
        return fail(QF_E_ARG, "qf_plan_grad_info: plan is NULL");
    if (sigma_passes)
        *sigma_passes = P->G == 0 ? 0 : P->n_ss_cls ? (int64_t)P->n_ss_cls : (int64_t)P->G;
    if (sweep_passes)
        *sweep_passes = P->adj_bits ? (int64_t)P->asegs.size() : (int64_t)P->runs.size();
    return QF_OK;
}

extern "C" int qf_plan_set_block_bits(qf_plan *P, int block_bits)
{
    return guarded([&]() -> int {
        if (!P)
            return fail(QF_E_ARG, "qf_plan_set_block_bits: plan is NULL");
        if (P->mem != qf_plan::kOwned)
            return fail(QF_E_ARG, "qf_plan_set_block_bits: an arena plan fixes its tiles at creation");
        set_block_bits(*P, block_bits);
        return QF_OK;
    });
}

extern "C" int qf_plan_apply_info(const qf_plan *P, int *block_bits, int64_t *runs, int64_t *passes)
{
    if (!P)
        return fail(QF_E_ARG, "qf_plan_apply_info: plan is NULL");
    if (block_bits)
        *block_bits = P->block_bits;
    if (runs)
        *runs = (int64_t)P->runs.size();
    if (passes)
        *passes = P->block_bits ? (int64_t)P->segs.size() : (int64_t)P->runs.size();
    return QF_OK;
}
