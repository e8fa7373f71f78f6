// Batched energy + adjoint gradient: many instances (molecules of uneven
// qubit count, or many parameter vectors) in ONE persistent kernel launch,
// optionally replayed as a HIP graph.
//
// Scheduling.  Instances are sorted by state size, largest first.  Instance
// e gets a team of W_e workgroups and the ticket range
// [ticket0_e, ticket0_e + W_e).  Every workgroup of the persistent grid takes
// tickets from one device counter; ticket t makes it member t - ticket0_e of
// the team of the instance that owns t.  A team runs the instance's passes
// (prepare and the run tables, each forward segment of runs on sub-cubes,
// sigma = H psi over output tiles by the streamed tile routine (512 threads of
// four outputs), each reverse segment) on disjoint parts of
// the state and meets at a team barrier after every pass:
// W = 1 teams only need the workgroup barrier, so small states stay in the
// CU's L2; larger teams use an agent-scope counter barrier with a bounded
// spin (timeout -> the instance's error flag, every wave still exits).  The
// grid never exceeds the resident capacity R and tickets are taken in order,
// so within one launch only the team being assembled waits for members, and
// every earlier team finishes and frees its workgroups for it.  When C
// persistent launches share the device (overlapping waves of a server),
// every team is capped at R / C workgroups: launches stuck at once would
// each hold fewer workgroups than their waiting team, less than R in total,
// so a free slot remains for one of them; a launch that completes its teams
// drains and releases its slots.  Either way the schedule cannot deadlock.
// A barrier that times out fails only its own instance: members stop
// waiting for each other, the instance's results are not published as
// valid, and the other instances of the launch complete normally.
//
// Reductions: each member sums its slice (wavefront shuffles + LDS), writes
// one partial per value, and member 0 sums the W partials in member order
// after the barrier, so an instance's results depend only on (instance, W):
// they are identical alone and in any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "qf_common.h"
#include "qf_host.h"
#include "qf_kernels.h"

namespace qf {

struct BatchEntry {
    int32_t n, W, nruns, G;
    uint32_t occ;
    int32_t run0;    // first RunDesc of the instance
    int32_t group0;  // first GroupDesc
    int32_t term0;   // first Hamiltonian string (GroupDesc ranges are instance-relative)
    int32_t theta0;  // first ansatz string (RunDesc.k0 is instance-relative)
    int32_t ticket0; // first ticket of the team
    int32_t part0;   // partial slots: W * K string sums, then W energy sums
    int32_t out;     // caller index of the instance
    int32_t K;       // ansatz strings of the instance
    int32_t aseg0, naseg, alr0;  // forward segments (Segment, LocalRun offsets)
    int32_t dseg0, ndseg, dlr0;  // reverse-sweep segments
    int32_t Bapp, Badj;          // their sub-cube sizes (qubits)
    int32_t cls0, ncls;          // streamed sigma sub-classes (SsCls), 0: untiled sigma
    int32_t word0, lo0;          // its group words and lo-terms
    int32_t imag;                // some string has an imaginary phase
    int32_t tabs0;               // the runs' (cos, sin) tables in the launch's table array
    uint64_t state0; // phi offset in amplitudes; lambda = phi + 2^n
};

// Team barrier across the XCDs of the chip. Each XCD has its own L2, and an
// agent-scope release writes back the whole L2 of the XCD that issues it, so
// the barrier pays it once per XCD the team spans instead of once per member:
// members on one XCD arrive on that XCD's counter after their stores have
// reached the shared L2, the last of them releases the L2 and arrives on the
// team counter, and everyone leaves when every spanned XCD has arrived.
// Counter words of a team (kSyncWords apart, zeroed before each launch):
//   [0] XCDs arrived (all epochs), [2 + x] members registered on XCD x,
//   [10 + x] arrivals on XCD x.
// A member's arrival on its XCD counter is not itself a release: its stores
// are complete in the XCD's L2 before it arrives (waitcnt + workgroup
// barrier), and the last arriver's release writes that L2 back to HBM.
constexpr int kSyncWords = 32;

__device__ __forceinline__ unsigned xcc_id()
{
    // hwreg(HW_REG_XCC_ID, offset 0, 4 bits): the XCD this wave runs on
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 7u;
}

struct TeamSync {
    unsigned *ctr;
    unsigned xcc;  // this member's XCD
    unsigned mine; // team members on it (0 until the first barrier has read the registration)
    unsigned nxcc; // XCDs the team spans
};

// bounded poll of a counter; on timeout or a raised error flag the caller
// goes on with whatever it has and the launch reports the error
__device__ __forceinline__ void spin_until(const unsigned *p, unsigned target, unsigned spin_limit, unsigned *err)
{
    unsigned spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        __builtin_amdgcn_s_sleep(4);
        if (++spins >= spin_limit) {
            atomicOr(err, 1u);
            return;
        }
    }
}

// thread 0 of each member, once per team and before its first barrier
__device__ __forceinline__ void team_register(int W, TeamSync &ts)
{
    if (W == 1)
        return;
    ts.xcc = xcc_id();
    ts.mine = 0;
    atomicAdd(ts.ctr + 2 + ts.xcc, 1u);
}

__device__ __forceinline__ void team_sync(int W, TeamSync &ts, unsigned epoch, unsigned spin_limit, unsigned *err)
{
    if (W == 1) {  // one workgroup: its waves share the CU's caches
        __syncthreads();
        return;
    }
    // every wave's stores have reached this XCD's L2 before thread 0 arrives
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!ts.mine) {
            // wait until all W members have registered, then read the census
            unsigned reg[8], spins = 0;
            for (;;) {
                unsigned tot = 0;
                for (int x = 0; x < 8; x++) {
                    reg[x] = __hip_atomic_load(ts.ctr + 2 + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    tot += reg[x];
                }
                if (tot >= (unsigned)W || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
                __builtin_amdgcn_s_sleep(4);
                if (++spins >= spin_limit) {
                    atomicOr(err, 1u);
                    break;
                }
            }
            unsigned nx = 0;
            for (int x = 0; x < 8; x++)
                nx += reg[x] ? 1u : 0u;
            ts.mine = max(1u, reg[ts.xcc]);
            ts.nxcc = max(1u, nx);
        }
        const unsigned old = atomicAdd(ts.ctr + 10 + ts.xcc, 1u);
        if (old + 1u == ts.mine * epoch) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(ts.ctr, 1u);
        }
        spin_until(ts.ctr, ts.nxcc * epoch, spin_limit, err);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Workgroup shape of the batched kernel: 512 threads, and LDS for one
// 2^12-amplitude sub-cube (blocked apply), one 2^11 sub-cube of each of phi
// and lambda (blocked adjoint) or the partner tile and the lo-term and group
// windows of the streamed sigma, two workgroups per CU.
constexpr int kBT = 512;
constexpr int kBW = kBT / 64;
constexpr int kSub = 4096;
static_assert(kBT == 512 && kSub >= (1 << kSsL) + kBT + kBT / 4,
              "the sigma tile and its lo-term and group windows fit the sub-cube image");
// pairs per thread in the common sub-cubes (2^12 forward, 2^11 reverse), which get unrolled variants
constexpr int kApplyPairs = kSub / 2 / kBT, kAdjPairs = kSub / 4 / kBT;
// runs of one forward segment (their fixed-bit parities in LDS; with the
// per-wave reverse-sweep sums this keeps the LDS image within two workgroups
// per CU); reverse segments hold at most kAdjRuns
constexpr int kBatchSegRuns = 128;

// member's slice [b, e) of `units`, in whole tiles of kBT * kItems
__device__ __forceinline__ void member_slice(uint64_t units, int W, int rank, uint64_t &b, uint64_t &e)
{
    const uint64_t per = (uint64_t)kBT * kItems;
    const uint64_t tiles = (units + per - 1) / per;
    const uint64_t tpm = (tiles + (uint64_t)W - 1) / (uint64_t)W;
    b = (uint64_t)rank * tpm * per;
    e = b + tpm * per;
    if (b > units)
        b = units;
    if (e > units)
        e = units;
}

__device__ void load_table(const RunDesc &d, const double *__restrict__ theta, double2 *tab)
{
    for (int u = threadIdx.x; u < (1 << d.r); u += kBT) {
        double th = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxRun; k++) {
            if (k < d.m) {
                const double v = (double)d.s[k] * theta[d.k0 + k];
                th += (__popc((uint32_t)u & d.e[k]) & 1) ? -v : v;
            }
        }
        double sn, cs;
        sincos(th, &sn, &cs);
        tab[u] = make_double2(cs, sn);
    }
    __syncthreads();
}

// (cos, sin) entries of one run from theta: entry u of run d goes to
// tab[d.tab + u] (the values load_table computes for that run)
__device__ void run_table(const RunDesc &d, const double *__restrict__ theta, double2 *tab)
{
    for (int u = threadIdx.x; u < (1 << d.r); u += kBT) {
        double th = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxRun; k++) {
            if (k < d.m) {
                const double v = (double)d.s[k] * theta[d.k0 + k];
                th += (__popc((uint32_t)u & d.e[k]) & 1) ? -v : v;
            }
        }
        double sn, cs;
        sincos(th, &sn, &cs);
        tab[d.tab + u] = make_double2(cs, sn);
    }
}

// offsets of the sub-cube's rows: the qubits of Q above q0, spread
__device__ void seg_hoff(const Segment &sg, uint32_t *hoff)
{
    if (threadIdx.x < (1u << sg.nhi)) {
        uint32_t o = 0;
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (q < sg.nhi)
                o |= ((threadIdx.x >> q) & 1u) << sg.hi[q];
        hoff[threadIdx.x] = o;
    }
}

// Apply a segment's runs to one 2^B sub-cube held in st (LDS).  Thread t's
// items are t + k * kBT (kBT = kItemStride); table indices and Z-parities
// split into the thread's part and the run's tabulated item parts, and the
// phase of a flip run folds into signs (rot_pair).
// NP > 0: exactly NP pairs per thread (NB = 2 NP kBT), all read before any
// is written so that their LDS reads are in flight together (the pairs are
// disjoint, which the compiler cannot tell); NP = 0: as many as NB holds.
template <bool SW, int NP>
__device__ __forceinline__ void sub_apply_pairs(double2 *st, const double2 *tb, const LocalRun &d, uint32_t NB,
                                                uint32_t yt, uint32_t ut, uint32_t pt31, uint32_t px31)
{
    if constexpr (NP > 0) {
        uint32_t y1[NP];
        double2 a[NP], b[NP], cs[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) {
            y1[k] = yt | insert0((uint32_t)k * kBT, d.hbit);
            cs[k] = tb[ut ^ (item_part(item_table(d), k) & 63u)];
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
    } else {
        for (uint32_t j = threadIdx.x, k = 0; j < NB / 2; j += kBT, k++) {
            const uint32_t ik = item_part(item_table(d), (int)k);
            const uint32_t y1 = yt | insert0(k * kBT, d.hbit), y2 = y1 ^ d.x;
            const double2 cs = tb[ut ^ (ik & 63u)];
            const uint32_t P1 = pt31 ^ ((ik >> 6) << 31);
            double2 a = st[y1], b = st[y2];
            rot_pair<SW>(cs.x, flip31(cs.y, P1), flip31(cs.y, P1 ^ px31), a, b);
            st[y1] = a;
            st[y2] = b;
        }
    }
}

// FIXNB: the sub-cube size when it is the common 2^12 (compile-time loops),
// 0 for 2^B
template <uint32_t FIXNB>
__device__ void sub_apply(double2 *__restrict__ psi, int B, uint32_t base, const Segment &sg,
                          const LocalRun *__restrict__ lr, const ApplyTriple *__restrict__ trip, const double2 *tab,
                          const uint32_t *hoff, double2 *st, uint32_t *pbzs)
{
    const uint32_t NB = FIXNB ? FIXNB : 1u << B, lomask = (1u << sg.q0) - 1u;
    // (the previous sub-cube's runs have all read pbzs: barrier before its write-back)
    sub_parities(lr, sg.r0, sg.r1 - sg.r0, base, pbzs, (int)threadIdx.x, kBT);
    __syncthreads();  // the previous sub-cube's LDS image is written back
    for (uint32_t l = threadIdx.x; l < NB; l += kBT)
        st[l] = psi[base | (l & lomask) | hoff[l >> sg.q0]];
    for (int ri = sg.r0; ri < sg.r1; ri++) {
        const LocalRun d = lr[ri];
        if constexpr (FIXNB == 8u * kBT) {
            // three runs per pass (ApplyTriple; flags in the flip runs' itm[1])
            if (d.x && (d.itm[1] & 1u)) {
                const ApplyTriple T = trip[ri];
                __syncthreads();
                apply_three<true>(st, tab, T, pbzs + (ri - sg.r0), threadIdx.x);
                ri += 2;
                continue;
            }
        }
        const double2 *tb = tab + (d.tab - sg.tab0);
        const uint32_t pbz = pbzs[ri - sg.r0];
        __syncthreads();
        if (d.x) {
            // rotation factor (-1)^p2 i^m with m = a0 + 3 (exp(-i theta P))
            const uint32_t m = (d.a0 + 3u) & 3u;
            const uint32_t yt = insert0(threadIdx.x, d.hbit);
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(yt, d.b, d.r);
            const uint32_t pt31 = (par(yt & d.z0) ^ (pbz >> 6) ^ (m >> 1)) << 31;
            const uint32_t px31 = par(d.x & d.z0) << 31;
            if (NB == 2u * kApplyPairs * kBT) {
                if (m & 1u)
                    sub_apply_pairs<true, kApplyPairs>(st, tb, d, NB, yt, ut, pt31, px31);
                else
                    sub_apply_pairs<false, kApplyPairs>(st, tb, d, NB, yt, ut, pt31, px31);
            } else if (m & 1u) {
                sub_apply_pairs<true, 0>(st, tb, d, NB, yt, ut, pt31, px31);
            } else {
                sub_apply_pairs<false, 0>(st, tb, d, NB, yt, ut, pt31, px31);
            }
        } else {
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(threadIdx.x, d.b, d.r);
            for (int k = 0; (uint32_t)k * kBT < NB; k++) {
                if (threadIdx.x + (uint32_t)k * kBT >= NB)
                    break;
                const uint32_t y = threadIdx.x | ((uint32_t)k * kBT);
                const double2 cs = tb[ut ^ item_part(item_table(d), k)];
                const double c = cs.x, s = cs.y;
                const double2 v = st[y];
                st[y] = make_double2(c * v.x + s * v.y, c * v.y - s * v.x);
            }
        }
    }
    __syncthreads();
    for (uint32_t l = threadIdx.x; l < NB; l += kBT)
        psi[base | (l & lomask) | hoff[l >> sg.q0]] = st[l];
}

// Reverse-sweep pairs of one flip run (q and the undo as in the single-
// instance blocked adjoint: rotation factor (-1)^p i^(a0 + 1), q the
// imaginary (a0 even) or real (a0 odd) part of the pair's bracket).
// NP as in sub_apply_pairs; the items' q reach accumulate(u_0, du, q)
// together when NP > 0 (du[k] = u_0 ^ u_k, uniform), one at a time otherwise.
template <bool SW, int NP, class Acc>
__device__ __forceinline__ void sub_adjoint_pairs(double2 *sp, double2 *sl, const double2 *tb, const LocalRun &d,
                                                  uint32_t NB, uint32_t yt, uint32_t ut, uint32_t pt31,
                                                  uint32_t px31, uint32_t dq31, Acc &&accumulate)
{
    const uint32_t i0 = item_part(item_table(d), 0) & 63u;
    uint32_t du[NP ? NP : 1];
    double qs[NP ? NP : 1];
    if constexpr (NP > 0) {
        // every item read before any is written, as in sub_apply_pairs
        uint32_t y1s[NP];
        double2 as[NP], bs[NP], las[NP], lbs[NP], css[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const uint32_t y1 = yt | insert0((uint32_t)k * kBT, d.hbit);
            y1s[k] = y1;
            css[k] = tb[ut ^ (item_part(item_table(d), k) & 63u)];
            as[k] = sp[y1];
            bs[k] = sp[y1 ^ d.x];
            las[k] = sl[y1];
            lbs[k] = sl[y1 ^ d.x];
        }
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const uint32_t ik = item_part(item_table(d), k);
            const uint32_t y1 = y1s[k], y2 = y1 ^ d.x;
            const uint32_t P1 = pt31 ^ ((ik >> 6) << 31), P2 = P1 ^ px31;
            double2 a = as[k], b = bs[k], la = las[k], lb = lbs[k];
            const double f1 = SW ? lb.x * a.y - lb.y * a.x : lb.x * a.x + lb.y * a.y;
            const double f2 = SW ? la.x * b.y - la.y * b.x : la.x * b.x + la.y * b.y;
            qs[k] = flip31(f1, P1 ^ dq31) + flip31(f2, P2 ^ dq31);
            du[k] = i0 ^ (ik & 63u);
            const double s1 = flip31(css[k].y, P1), s2 = flip31(css[k].y, P2);
            rot_pair<SW>(css[k].x, s1, s2, a, b);
            rot_pair<SW>(css[k].x, s1, s2, la, lb);
            sp[y1] = a;
            sp[y2] = b;
            sl[y1] = la;
            sl[y2] = lb;
        }
        accumulate(ut ^ i0, du, qs);
    } else {
        for (uint32_t j = threadIdx.x, k = 0; j < NB / 2; j += kBT, k++) {
            const uint32_t ik = item_part(item_table(d), (int)k);
            const uint32_t y1 = yt | insert0(k * kBT, d.hbit), y2 = y1 ^ d.x;
            const uint32_t u = ut ^ (ik & 63u);
            const double2 cs = tb[u];
            const uint32_t P1 = pt31 ^ ((ik >> 6) << 31), P2 = P1 ^ px31;
            double2 a = sp[y1], b = sp[y2], la = sl[y1], lb = sl[y2];
            const double f1 = SW ? lb.x * a.y - lb.y * a.x : lb.x * a.x + lb.y * a.y;
            const double f2 = SW ? la.x * b.y - la.y * b.x : la.x * b.x + la.y * b.y;
            const double q = flip31(f1, P1 ^ dq31) + flip31(f2, P2 ^ dq31);
            const double s1 = flip31(cs.y, P1), s2 = flip31(cs.y, P2);
            rot_pair<SW>(cs.x, s1, s2, a, b);
            rot_pair<SW>(cs.x, s1, s2, la, lb);
            sp[y1] = a;
            sp[y2] = b;
            sl[y1] = la;
            sl[y2] = lb;
            const uint32_t d1[1] = {0u};
            const double q1[1] = {q};
            accumulate(u, d1, q1);
        }
    }
}

// Undo a segment's runs (last first) on one 2^B sub-cube of phi (sp) and
// lambda (sl); before a run is undone each wave adds the run's 8 sums of
// 2 Im <lambda|P_k|phi> / 2 over the sub-cube (Walsh sums, or per string for
// rank > 3) to its own slots wred[wave][run] (no barrier, no cross-wave step
// per run; the member sums the waves once per segment).
// FIXNB: the sub-cube size when it is the common 2^11, 0 for 2^B
template <uint32_t FIXNB>
__device__ void sub_adjoint(double2 *__restrict__ phi, double2 *__restrict__ lam, int B, uint32_t base,
                            const Segment &sg, const LocalRun *__restrict__ lr, const AdjPair *__restrict__ apairs,
                            const double2 *tab, const uint32_t *hoff, double2 *sp, double2 *sl,
                            double (*wred)[kAdjRuns][kMaxRun], uint32_t *pbzs)
{
    const uint32_t NB = FIXNB ? FIXNB : 1u << B, lomask = (1u << sg.q0) - 1u;
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    sub_parities(lr, sg.r0, sg.r1 - sg.r0, base, pbzs, (int)threadIdx.x, kBT);
    __syncthreads();  // the previous sub-cube's LDS images are written back
    for (uint32_t l = threadIdx.x; l < NB; l += kBT) {
        const uint32_t y = base | (l & lomask) | hoff[l >> sg.q0];
        sp[l] = phi[y];
        sl[l] = lam[y];
    }
    for (int ri = sg.r1 - 1; ri >= sg.r0; ri--) {
        if constexpr (FIXNB == 4u * kBT) {
            // two runs per pass (AdjPair)
            const AdjPair pr = apairs[ri];
            if (pr.w0 & 1u) {
                const uint32_t pbzA = pbzs[ri - sg.r0], pbzB = pbzs[ri - 1 - sg.r0];
                __syncthreads();  // the previous run's updates are visible
                adjoint_two<true>(sp, sl, tab, pr, pbzA, pbzB, threadIdx.x, lane, wred[wave][ri - sg.r0],
                                  wred[wave][ri - 1 - sg.r0]);
                ri--;
                continue;
            }
        }
        const LocalRun d = lr[ri];
        const double2 *tb = tab + (d.tab - sg.tab0);
        const uint32_t pbz = pbzs[ri - sg.r0];
        // string k's weight is s_k (-1)^popcount(u & e_k): for rank <= 3 the
        // pass sums the 8 Walsh terms (-1)^popcount(u & e) q and string k
        // takes s_k times term e_k; otherwise acc[k] is string k's own sum
        const bool walsh = d.r <= 3;
        double acc[kMaxRun];
#pragma unroll
        for (int k = 0; k < kMaxRun; k++)
            acc[k] = -0.0;  // -0.0 + x is x, so the first term needs no add
        // items i of the thread have table indices u0 ^ du[i] (du uniform)
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
        __syncthreads();  // the previous run's updates are visible
        if (d.x) {
            const uint32_t m = (d.a0 + 1u) & 3u;
            const uint32_t yt = insert0(threadIdx.x, d.hbit);
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(yt, d.b, d.r);
            const uint32_t pt31 = (par(yt & d.z0) ^ (pbz >> 6) ^ (m >> 1)) << 31;
            const uint32_t px31 = par(d.x & d.z0) << 31;
            const uint32_t dq31 = ((d.a0 >> 1) ^ (m >> 1)) << 31;
            if (NB == 2u * kAdjPairs * kBT) {
                if (m & 1u)
                    sub_adjoint_pairs<true, kAdjPairs>(sp, sl, tb, d, NB, yt, ut, pt31, px31, dq31, accumulate);
                else
                    sub_adjoint_pairs<false, kAdjPairs>(sp, sl, tb, d, NB, yt, ut, pt31, px31, dq31, accumulate);
            } else if (m & 1u) {
                sub_adjoint_pairs<true, 0>(sp, sl, tb, d, NB, yt, ut, pt31, px31, dq31, accumulate);
            } else {
                sub_adjoint_pairs<false, 0>(sp, sl, tb, d, NB, yt, ut, pt31, px31, dq31, accumulate);
            }
        } else {
            const uint32_t ut = (pbz & 63u) ^ gf2_coords(threadIdx.x, d.b, d.r);
            for (int k = 0; (uint32_t)k * kBT < NB; k++) {
                if (threadIdx.x + (uint32_t)k * kBT >= NB)
                    break;
                const uint32_t y = threadIdx.x | ((uint32_t)k * kBT);
                const uint32_t u = ut ^ item_part(item_table(d), k);
                const double2 cs = tb[u];
                const double c = cs.x, s = cs.y;
                const double2 a = sp[y], la = sl[y];
                const double q = la.x * a.y - la.y * a.x;
                sp[y] = make_double2(c * a.x - s * a.y, c * a.y + s * a.x);
                sl[y] = make_double2(c * la.x - s * la.y, c * la.y + s * la.x);
                const uint32_t d1[1] = {0u};
                const double q1[1] = {q};
                accumulate(u, d1, q1);
            }
        }
        {
            const double h = wave_sum8(acc, lane);
            if (sum8_writer(lane))
                wave_add(&wred[wave][ri - sg.r0][sum8_index(lane)], h);
        }
    }
    __syncthreads();
    for (uint32_t l = threadIdx.x; l < NB; l += kBT) {
        const uint32_t y = base | (l & lomask) | hoff[l >> sg.q0];
        phi[y] = sp[l];
        lam[y] = sl[l];
    }
}

template <int M> __device__ void block_sum(double (&v)[M], double *out)
{
    __shared__ double lds[kBW][kMaxRun];
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
        for (int w = 0; w < kBW; w++)
            s += lds[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

__device__ void pass_prepare(double2 *__restrict__ psi, uint64_t b, uint64_t e, uint32_t occ)
{
    for (uint64_t y = b + threadIdx.x; y < e; y += kBT)
        psi[y] = make_double2(y == occ ? 1.0 : 0.0, 0.0);
}

__device__ void pass_apply(double2 *__restrict__ psi, const RunDesc &d, const double2 *tab, uint64_t b,
                           uint64_t e)
{
    const uint64_t per = (uint64_t)kBT * kItems;
    const bool diag = d.x == 0;
    for (uint64_t j0 = b; j0 < e; j0 += per) {
        uint32_t y[kItems];
        double2 a[kItems], c2[kItems];
        bool ok[kItems];
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t j = j0 + threadIdx.x + (uint64_t)i * kBT;
            ok[i] = j < e;
            const uint32_t jj = (uint32_t)(ok[i] ? j : b);
            y[i] = diag ? jj : insert0(jj, d.hbit);
            a[i] = psi[y[i]];
            c2[i] = psi[y[i] ^ d.x];
        }
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            if (!ok[i])
                continue;
            const uint32_t y1 = y[i], y2 = y1 ^ d.x;
            const double2 cs = tab[run_coords(d, y1)];
            const double c = cs.x, s = cs.y;
            if (diag) {
                psi[y1] = make_double2(c * a[i].x + s * a[i].y, c * a[i].y - s * a[i].x);
            } else {
                const double2 pb = mul_ik((d.a0 + 2u * par(y2 & d.z0)) & 3u, c2[i]);
                const double2 pa = mul_ik((d.a0 + 2u * par(y1 & d.z0)) & 3u, a[i]);
                psi[y1] = make_double2(c * a[i].x + s * pb.y, c * a[i].y - s * pb.x);
                psi[y2] = make_double2(c * c2[i].x + s * pa.y, c * c2[i].y - s * pa.x);
            }
        }
    }
}

__device__ double pass_sigma(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                             const GroupDesc *__restrict__ groups, int G, const uint32_t *__restrict__ zs,
                             const double *__restrict__ cs, uint64_t b, uint64_t e)
{
    const uint64_t per = (uint64_t)kBT * kItems;
    double acc = 0.0;
    for (uint64_t j0 = b; j0 < e; j0 += per) {
        uint32_t y[kItems];
        bool ok[kItems];
        double2 l[kItems];
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t j = j0 + threadIdx.x + (uint64_t)i * kBT;
            ok[i] = j < e;
            y[i] = (uint32_t)(ok[i] ? j : b);
            l[i] = make_double2(0.0, 0.0);
        }
        for (int gi = 0; gi < G; gi++) {
            const GroupDesc g = groups[gi];
            uint32_t y2[kItems];
            double2 bv[kItems];
#pragma unroll
            for (int i = 0; i < kItems; i++) {
                y2[i] = y[i] ^ g.x;
                bv[i] = psi[y2[i]];
            }
            double dre[kItems], dim[kItems];
            static_assert(kItems == 4 && kBT == 512, "items are y0 + 512 i, i < 4");
            group_d4<9>(g, zs, cs, (uint32_t)(j0 + threadIdx.x) ^ g.x, dre, dim);
            if (g.k1 > g.kre) {
#pragma unroll
                for (int i = 0; i < kItems; i++) {
                    l[i].x += dre[i] * bv[i].x - dim[i] * bv[i].y;
                    l[i].y += dre[i] * bv[i].y + dim[i] * bv[i].x;
                }
            } else {  // real phases only
#pragma unroll
                for (int i = 0; i < kItems; i++) {
                    l[i].x += dre[i] * bv[i].x;
                    l[i].y += dre[i] * bv[i].y;
                }
            }
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
    return acc;
}

__device__ void pass_adjoint(double2 *__restrict__ phi, double2 *__restrict__ lam, const RunDesc &d,
                             const double2 *tab, uint64_t b, uint64_t e, double (&acc)[kMaxRun])
{
    const uint64_t per = (uint64_t)kBT * kItems;
    const bool diag = d.x == 0;
    for (uint64_t j0 = b; j0 < e; j0 += per) {
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t j = j0 + threadIdx.x + (uint64_t)i * kBT;
            if (j >= e)
                break;
            const uint32_t y1 = diag ? (uint32_t)j : insert0((uint32_t)j, d.hbit);
            const uint32_t y2 = y1 ^ d.x;
            const double2 a = phi[y1], la = lam[y1];
            const uint32_t u = run_coords(d, y1);
            const double2 cs = tab[u];
            const double c = cs.x, s = cs.y;
            double q;
            if (diag) {
                q = la.x * a.y - la.y * a.x;
                phi[y1] = make_double2(c * a.x - s * a.y, c * a.y + s * a.x);
                lam[y1] = make_double2(c * la.x - s * la.y, c * la.y + s * la.x);
            } else {
                const double2 bb = phi[y2], lb = lam[y2];
                const uint32_t k1 = (d.a0 + 2u * par(y1 & d.z0)) & 3u;
                const uint32_t k2 = (d.a0 + 2u * par(y2 & d.z0)) & 3u;
                const double2 wa = mul_ik(k1, a), wb = mul_ik(k2, bb);
                q = (lb.x * wa.y - lb.y * wa.x) + (la.x * wb.y - la.y * wb.x);
                phi[y1] = make_double2(c * a.x - s * wb.y, c * a.y + s * wb.x);
                phi[y2] = make_double2(c * bb.x - s * wa.y, c * bb.y + s * wa.x);
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
}

__global__ void k_batch_reset(unsigned *sync, int nentries, unsigned *ticket, unsigned *err)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nentries * kSyncWords; i += gridDim.x * blockDim.x)
        sync[i] = 0u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nentries; i += gridDim.x * blockDim.x)
        err[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *ticket = 0u;
}

__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(const BatchEntry *__restrict__ entries, int nentries,
                                               unsigned total_tickets, const RunDesc *__restrict__ runs,
                                               const Segment *__restrict__ segs, const LocalRun *__restrict__ lruns,
                                               const ApplyTriple *__restrict__ atrip,
                                               const AdjPair *__restrict__ apairs,
                                               const uint32_t *__restrict__ smap,
                                               const GroupDesc *__restrict__ groups,
                                               const SsCls *__restrict__ sscls, const uint32_t *__restrict__ sswords,
                                               const SsLo *__restrict__ sslos, double2 *__restrict__ tabs,
                                               const uint32_t *__restrict__ zs,
                                               const double *__restrict__ cs, const double *__restrict__ theta,
                                               double2 *states, double *partials, unsigned *sync, unsigned *ticket,
                                               unsigned *err, double *E_out, double *grad_out, unsigned spin_limit,
                                               double *mb_E, double *mb_grad, unsigned *mb_flag)
{
    __shared__ int s_entry, s_rank;
    __shared__ double2 s_sub[kSub];
    __shared__ double2 s_tab[kAdjTab];
    __shared__ uint32_t s_hoff[64];
    __shared__ double s_wred[kBW][kAdjRuns][kMaxRun];  // per-wave run sums of a reverse segment
    __shared__ double s_part[kMaxRun];
    __shared__ uint32_t s_pbz[kBatchSegRuns];
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned t = atomicAdd(ticket, 1u);
            int e = -1, rank = 0;
            if (t < total_tickets) {
                int lo = 0, hi = nentries - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((unsigned)entries[mid].ticket0 <= t)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                e = lo;
                rank = (int)(t - (unsigned)entries[lo].ticket0);
            }
            s_entry = e;
            s_rank = rank;
        }
        __syncthreads();
        // uniform across the workgroup: scalar registers, so that the entry
        // and every descriptor reached from it are scalar loads
        const int ei = __builtin_amdgcn_readfirstlane(s_entry), rank = __builtin_amdgcn_readfirstlane(s_rank);
        __syncthreads();
        if (ei < 0)
            break;
        const BatchEntry en = entries[ei];
        const int W = en.W, n = en.n;
        const uint64_t dim = 1ull << n;
        double2 *phi = states + en.state0;
        double2 *lam = phi + dim;
        const double *th = theta + en.theta0;
        double *gpart = partials + en.part0;     // [W][K] string sums
        double *epart = gpart + (size_t)W * en.K; // [W] energy sums
        unsigned *ierr = err + ei;  // this instance's error flag
        TeamSync ts;
        ts.ctr = sync + (size_t)ei * kSyncWords;
        if (threadIdx.x == 0)
            team_register(W, ts);
        unsigned epoch = 0;
        uint64_t b, e;

        member_slice(dim, W, rank, b, e);
        pass_prepare(phi, b, e, en.occ);
        // the runs' (cos, sin) tables, once per launch (runs rank, rank + W, ...)
        for (int r = rank; r < en.nruns; r += W)
            run_table(runs[en.run0 + r], th, tabs + en.tabs0);
        team_sync(W, ts, ++epoch, spin_limit, ierr);

        // forward: segments of runs on sub-cubes, members take sub-cubes rank, rank + W, ...
        for (int si = 0; si < en.naseg; si++) {
            const Segment sg = segs[en.aseg0 + si];
            if (!sg.Q) {
                const RunDesc d = runs[en.run0 + sg.r0];
                load_table(d, th, s_tab);
                member_slice(d.x ? dim >> 1 : dim, W, rank, b, e);
                pass_apply(phi, d, s_tab, b, e);
            } else {
                const LocalRun *lr = lruns + en.alr0;
                for (int t = (int)threadIdx.x; t < sg.ntab; t += kBT)
                    s_tab[t] = tabs[en.tabs0 + sg.tab0 + t];
                seg_hoff(sg, s_hoff);
                const uint32_t nsub = 1u << (n - en.Bapp);
                for (uint32_t sc = (uint32_t)rank; sc < nsub; sc += (uint32_t)W) {
                    const uint32_t base = subcube_base(sc, sg);
                    if (en.Bapp == 12)
                        sub_apply<(uint32_t)kSub>(phi, en.Bapp, base, sg, lr, atrip + en.alr0, s_tab, s_hoff, s_sub,
                                                  s_pbz);
                    else
                        sub_apply<0>(phi, en.Bapp, base, sg, lr, atrip + en.alr0, s_tab, s_hoff, s_sub, s_pbz);
                }
            }
            team_sync(W, ts, ++epoch, spin_limit, ierr);
        }

        {
            double v[1] = {0.0};
            if (en.ncls) {
                // output tiles rank, rank + W, ... (a team has at most one member
                // per tile); the tile and its windows live in the sub-cube image
                double2 *tile = s_sub;
                uint4 *wlo = reinterpret_cast<uint4 *>(s_sub + (1u << kSsL));
                uint32_t *wgw = reinterpret_cast<uint32_t *>(s_sub + (1u << kSsL) + kBT);
                if (en.imag)
                    v[0] = sigma_stream<kBT, true>(phi, lam, (uint32_t)rank, (uint32_t)W, 1u << (n - kSsL),
                                                   sscls + en.cls0, en.ncls, sswords + en.word0, sslos + en.lo0,
                                                   tile, wlo, wgw);
                else
                    v[0] = sigma_stream<kBT, false>(phi, lam, (uint32_t)rank, (uint32_t)W, 1u << (n - kSsL),
                                                    sscls + en.cls0, en.ncls, sswords + en.word0, sslos + en.lo0,
                                                    tile, wlo, wgw);
            } else {
                member_slice(dim, W, rank, b, e);
                v[0] = pass_sigma(phi, lam, groups + en.group0, en.G, zs + en.term0, cs + en.term0, b, e);
            }
            block_sum<1>(v, s_part);
            if (threadIdx.x == 0)
                epart[rank] = s_part[0];
        }
        team_sync(W, ts, ++epoch, spin_limit, ierr);

        // reverse sweep: segments last first; each member leaves its string sums in gpart[rank]
        for (int si = en.ndseg - 1; si >= 0; si--) {
            const Segment sg = segs[en.dseg0 + si];
            if (!sg.Q) {
                const RunDesc d = runs[en.run0 + sg.r0];
                load_table(d, th, s_tab);
                member_slice(d.x ? dim >> 1 : dim, W, rank, b, e);
                double acc[kMaxRun];
#pragma unroll
                for (int k = 0; k < kMaxRun; k++)
                    acc[k] = 0.0;
                pass_adjoint(phi, lam, d, s_tab, b, e, acc);
                block_sum<kMaxRun>(acc, s_part);
                if (threadIdx.x < (uint32_t)d.m)
                    gpart[(size_t)rank * en.K + d.k0 + threadIdx.x] = s_part[threadIdx.x];
            } else {
                const LocalRun *lr = lruns + en.dlr0;
                const int sk0 = lr[sg.r0].k0;
                const int nstr = lr[sg.r1 - 1].k0 + lr[sg.r1 - 1].m - sk0;
                for (int t = (int)threadIdx.x; t < sg.ntab; t += kBT)
                    s_tab[t] = tabs[en.tabs0 + sg.tab0 + t];
                seg_hoff(sg, s_hoff);
                for (int t = (int)threadIdx.x; t < kBW * kAdjRuns * kMaxRun; t += kBT)
                    (&s_wred[0][0][0])[t] = 0.0;
                const uint32_t nsub = 1u << (n - en.Badj);
                for (uint32_t sc = (uint32_t)rank; sc < nsub; sc += (uint32_t)W) {
                    const uint32_t base = subcube_base(sc, sg);
                    if (en.Badj == 11)
                        sub_adjoint<(uint32_t)kSub / 2>(phi, lam, en.Badj, base, sg, lr, apairs + en.dlr0, s_tab,
                                                        s_hoff, s_sub, s_sub + (kSub / 2), s_wred, s_pbz);
                    else
                        sub_adjoint<0>(phi, lam, en.Badj, base, sg, lr, apairs + en.dlr0, s_tab, s_hoff, s_sub,
                                       s_sub + (kSub / 2), s_wred, s_pbz);
                }
                // the waves' sums in wave order; smap: each string's run,
                // Walsh column (or string index) and sign
                __syncthreads();
                for (int t = (int)threadIdx.x; t < nstr; t += kBT) {
                    const uint32_t m = smap[en.theta0 + sk0 + t];
                    double v = 0.0;
#pragma unroll
                    for (int w = 0; w < kBW; w++)
                        v += s_wred[w][m >> 4][m & 7u];
                    gpart[(size_t)rank * en.K + sk0 + t] = (m & 8u) ? -v : v;
                }
            }
            team_sync(W, ts, ++epoch, spin_limit, ierr);
        }
        if (rank == 0) {
            for (int k = threadIdx.x; k < en.K; k += kBT) {
                double s = 0.0;
                for (int w = 0; w < W; w++)
                    s += gpart[(size_t)w * en.K + k];
                grad_out[en.theta0 + k] = 2.0 * s;
            }
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int w = 0; w < W; w++)
                    s += epart[w];
                E_out[en.out] = s;
                if (mb_E)
                    mb_E[en.out] = s;
            }
            if (mb_flag) {
                // per-instance completion: results to host memory, then the
                // flag (1: valid; 2: a barrier of this instance timed out)
                __syncthreads();
                for (int k = threadIdx.x; k < en.K; k += kBT)
                    mb_grad[en.theta0 + k] = grad_out[en.theta0 + k];
                __threadfence_system();
                __syncthreads();
                if (threadIdx.x == 0) {
                    const unsigned bad = __hip_atomic_load(ierr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&mb_flag[en.out], bad ? 2u : 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        __syncthreads();
    }
}

} // namespace qf

struct qf_batch {
    int count = 0;
    int nentries = 0;
    unsigned total_tickets = 0;
    unsigned grid = 0;
    unsigned spin_limit = 1u << 28;
    bool owns_device = true;  // false: device data lives in a caller arena
    void *d_base = nullptr;   // the one device allocation of an owning batch
    int64_t K_total = 0;
    std::vector<int64_t> koff;  // caller-order offsets into theta / grad
    std::vector<int> W;         // per caller instance
    std::vector<int> status;    // per caller instance, from the last collected launch
    std::vector<int> entry_out; // caller index of each entry (launch order)
    std::vector<int> nq;
    size_t state_bytes = 0;
    size_t device_bytes = 0;
    // device data (owned or carved from the arena)
    qf::BatchEntry *d_entries = nullptr;
    qf::RunDesc *d_runs = nullptr;
    qf::Segment *d_segs = nullptr;
    qf::LocalRun *d_lruns = nullptr;
    qf::GroupDesc *d_groups = nullptr;
    qf::SsCls *d_sscls = nullptr;
    uint32_t *d_sswords = nullptr;
    qf::SsLo *d_sslos = nullptr;
    qf::ApplyTriple *d_atrip = nullptr;
    qf::AdjPair *d_apairs = nullptr;
    uint32_t *d_smap = nullptr;
    double2 *d_tabs = nullptr;  // (cos, sin) tables of every instance's runs, filled in the launch
    uint32_t *d_z = nullptr;
    double *d_c = nullptr;
    double *d_theta = nullptr;
    double2 *d_states = nullptr;
    double *d_partials = nullptr;
    unsigned *d_sync = nullptr;
    unsigned *d_ticket = nullptr;
    unsigned *d_err = nullptr;
    double *d_E = nullptr;
    double *d_grad = nullptr;
    // host side
    std::vector<double> theta_host;  // arena mode: source of the async theta upload
    double *h_theta = nullptr;       // owned mode: pinned staging (graph-capturable copies)
    double *h_E = nullptr;
    double *h_grad = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    double *mb_E = nullptr;  // mailbox of the current launch (host, coherent), or null
    double *mb_grad = nullptr;
    unsigned *mb_flag = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;

    void drop_graph()
    {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }

    ~qf_batch()
    {
        drop_graph();
        if (done)
            (void)hipEventDestroy(done);
        void *hp[] = {h_theta, h_E, h_grad};
        for (void *p : hp)
            if (p)
                (void)hipHostFree(p);
        if (owns_device && d_base)
            (void)hipFree(d_base);
    }
};

namespace qf {

int default_team(int n)
{
    int w = n >= 14 ? 1 << (n - 14) : 1;
    return std::min(w, 256);
}

unsigned resident_grid()
{
    int dev = 0, cus = 0, per = 0;
    QF_HIP(hipGetDevice(&dev));
    QF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    QF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(k_batch), kBT, 0));
    if (per < 1)
        per = 1;
    return (unsigned)(cus * per);
}

// Host tables of a batch in launch order (largest instance first).
struct BatchHost {
    std::vector<BatchEntry> ent;
    std::vector<RunDesc> runs;
    std::vector<Segment> segs;
    std::vector<LocalRun> lruns;
    std::vector<ApplyTriple> atrip;  // parallel to lruns: forward three-run passes
    std::vector<AdjPair> apairs;     // parallel to lruns: reverse two-run passes
    std::vector<uint32_t> smap;      // per ansatz string (caller offsets): run, column, sign
    std::vector<GroupDesc> groups;
    std::vector<SsCls> sscls;
    std::vector<uint32_t> sswords;
    std::vector<SsLo> sslos;
    std::vector<uint32_t> zs;
    std::vector<double> cs;
    uint64_t state_amps = 0;
    int64_t tickets = 0, parts = 0, tabs = 0;
};

// Team sizes W[i] on a resident grid of `grid` workgroups shared by up to
// `concurrent` persistent launches: team[i] > 0 asks for that many, 0 (or
// team == NULL) for the built-in table; team[i] < 0 shares the grid by
// work, 2^n (K + Hamiltonian strings), among the instances that ask for it,
// with at least -team[i] members and at most one forward sub-cube (2^12
// amplitudes) per member.  Every team is then clamped to one reverse-sweep
// sub-cube (2^11 amplitudes) per member and to grid / concurrent.
void team_sizes(int count, const int *n_qubits, const int64_t *K, const int64_t *strings, const int *team,
                unsigned grid, int concurrent, int *W)
{
    for (int i = 0; i < count; i++)
        W[i] = (team && team[i] > 0) ? team[i] : default_team(n_qubits[i]);
    if (team) {
        double total = 0.0;
        for (int i = 0; i < count; i++)
            if (team[i] < 0)
                total += std::ldexp((double)(K[i] + strings[i]), n_qubits[i]);
        for (int i = 0; i < count; i++)
            if (team[i] < 0) {
                // a shared team takes at most one forward sub-cube per member:
                // more members mostly add barrier traffic
                const double w = std::ldexp((double)(K[i] + strings[i]), n_qubits[i]);
                const double cap = std::ldexp(1.0, std::max(0, n_qubits[i] - 12));
                const int share = (int)std::min<double>({(double)grid, cap, std::floor((double)grid * w / total)});
                W[i] = std::max(-team[i], share);
            }
    }
    const int64_t per_launch = std::max<int64_t>(1, (int64_t)grid / std::max(1, concurrent));
    for (int i = 0; i < count; i++) {
        const int n = n_qubits[i];
        const int64_t tiles = std::max<int64_t>(1, (int64_t)(1ull << (n - 1)) / 1024);
        W[i] = (int)std::min<int64_t>({(int64_t)W[i], tiles, per_launch});
    }
}

// Validate the instances, pick team sizes and assemble the host tables.
void batch_assemble(qf_batch &B, BatchHost &T, int count, const int *n_qubits, const uint64_t *occ_mask,
                    const qf_term *const *A, const int64_t *K, const qf_term *const *H,
                    const int64_t *const *group_off, const int64_t *n_groups, const int *team, int concurrent = 1)
{
    if (count < 1 || !n_qubits || !occ_mask || !K || !A || !H || !group_off || !n_groups)
        raise(QF_E_ARG, "qf_batch_create: null array or count < 1");
    B.count = count;
    B.koff.assign((size_t)count + 1, 0);
    B.W.assign((size_t)count, 1);
    B.nq.assign((size_t)count, 0);
    for (int i = 0; i < count; i++) {
        const int n = n_qubits[i];
        if (n < 1 || n > 30)
            raise(QF_E_RANGE, "instance " + std::to_string(i) + ": n_qubits out of range [1, 30]");
        if (occ_mask[i] >> n)
            raise(QF_E_RANGE, "instance " + std::to_string(i) + ": occ_mask has a bit >= n_qubits");
        if (K[i] < 0 || n_groups[i] < 1 || (K[i] > 0 && !A[i]) || !H[i] || !group_off[i])
            raise(QF_E_ARG, "instance " + std::to_string(i) + ": bad ansatz or Hamiltonian");
        B.koff[(size_t)i + 1] = B.koff[(size_t)i] + K[i];
        B.nq[(size_t)i] = n;
        if (group_off[i][n_groups[i]] < 0)
            raise(QF_E_ARG, "instance " + std::to_string(i) + ": bad group offsets");
    }
    B.K_total = B.koff[(size_t)count];
    B.grid = resident_grid();
    std::vector<int64_t> strings((size_t)count);
    for (int i = 0; i < count; i++)
        strings[(size_t)i] = group_off[i][n_groups[i]];
    team_sizes(count, n_qubits, K, strings.data(), team, B.grid, concurrent, B.W.data());
    std::vector<int> order((size_t)count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return B.nq[a] > B.nq[b]; });
    T.smap.assign((size_t)std::max<int64_t>(B.K_total, 1), 0u);
    for (int i : order) {
        const int n = n_qubits[i];
        int tab = 0;
        std::vector<RunDesc> r;
        if (K[i] > 0) {
            check_terms("batch ansatz", n, A[i], K[i]);
            r = make_runs(A[i], K[i], tab);
        }
        std::vector<GroupDesc> gd;
        std::vector<uint32_t> z;
        std::vector<double> c;
        build_groups(n, H[i], group_off[i], n_groups[i], gd, z, c);
        std::vector<SsCls> ssc;
        std::vector<uint32_t> ssw;
        std::vector<SsLo> ssl;
        if (n > kSsL && !gd.empty())
            sigma_stream_tables(gd, z, c, kBT, ssc, ssw, ssl);
        // forward segments on 2^min(n,12) sub-cubes, reverse on 2^min(n,11)
        // (phi and lambda share the LDS image)
        const int Bapp = std::min(n, 12), Badj = std::min(n, 11);
        std::vector<Segment> sa, sd;
        std::vector<LocalRun> la, ld;
        if (!r.empty()) {
            build_segments(r, n, Bapp, std::min(6, Bapp), sa, la, kBatchSegRuns, kAdjTab);
            build_segments(r, n, Badj, std::min(6, Badj), sd, ld, kAdjRuns, kAdjTab);
        }
        // multi-run passes on the full-size sub-cubes: three runs forward
        // (flags in the flip runs' itm[1]), two runs in the reverse sweep
        std::vector<ApplyTriple> at(la.size());
        std::memset(at.data(), 0, at.size() * sizeof(ApplyTriple));
        if (Bapp == 12 && !la.empty()) {
            at = apply_triples(sa, la);
            for (size_t j = 0; j < la.size(); j++)
                if (la[j].x)
                    la[j].itm[1] = at[j].w0 & 3u;
        }
        std::vector<AdjPair> ap(ld.size());
        std::memset(ap.data(), 0, ap.size() * sizeof(AdjPair));
        if (Badj == 11 && !ld.empty())
            ap = adjoint_pairs(sd, ld);
        // string k of reverse-segment run r: Walsh column e_k (rank <= 3) or
        // k, the sign of s_k, r within its segment (at the caller's offset)
        for (const Segment &sg : sd) {
            if (!sg.Q)
                continue;
            for (int rr = sg.r0; rr < sg.r1; rr++) {
                const LocalRun &L = ld[(size_t)rr];
                const bool walsh = L.r <= 3;
                for (int k = 0; k < L.m; k++)
                    T.smap[(size_t)(B.koff[(size_t)i] + L.k0 + k)] =
                        (uint32_t)(walsh ? L.e[k] : k) | (walsh && L.s[k] < 0 ? 8u : 0u) | (uint32_t)(rr - sg.r0) << 4;
            }
        }
        BatchEntry e;
        std::memset(&e, 0, sizeof e);
        e.n = n;
        e.Bapp = Bapp;
        e.Badj = Badj;
        e.aseg0 = (int32_t)T.segs.size();
        e.naseg = (int32_t)sa.size();
        e.alr0 = (int32_t)T.lruns.size();
        e.dseg0 = e.aseg0 + e.naseg;
        e.ndseg = (int32_t)sd.size();
        e.dlr0 = e.alr0 + (int32_t)la.size();
        T.segs.insert(T.segs.end(), sa.begin(), sa.end());
        T.segs.insert(T.segs.end(), sd.begin(), sd.end());
        T.lruns.insert(T.lruns.end(), la.begin(), la.end());
        T.lruns.insert(T.lruns.end(), ld.begin(), ld.end());
        T.atrip.insert(T.atrip.end(), at.begin(), at.end());
        T.atrip.resize(T.lruns.size());
        T.apairs.resize(T.lruns.size() - ld.size());
        T.apairs.insert(T.apairs.end(), ap.begin(), ap.end());
        e.W = B.W[(size_t)i];
        e.nruns = (int32_t)r.size();
        e.G = (int32_t)gd.size();
        e.occ = (uint32_t)occ_mask[i];
        e.run0 = (int32_t)T.runs.size();
        e.group0 = (int32_t)T.groups.size();
        e.term0 = (int32_t)T.zs.size();
        e.cls0 = (int32_t)T.sscls.size();
        e.ncls = (int32_t)ssc.size();
        e.word0 = (int32_t)T.sswords.size();
        e.lo0 = (int32_t)T.sslos.size();
        e.imag = 0;
        for (const GroupDesc &g : gd)
            if (g.k1 > g.kre)
                e.imag = 1;
        e.tabs0 = (int32_t)T.tabs;
        e.theta0 = (int32_t)B.koff[(size_t)i];
        e.ticket0 = (int32_t)T.tickets;
        e.part0 = (int32_t)T.parts;
        e.out = i;
        e.K = (int32_t)K[i];
        e.state0 = T.state_amps;
        T.ent.push_back(e);
        T.runs.insert(T.runs.end(), r.begin(), r.end());
        T.groups.insert(T.groups.end(), gd.begin(), gd.end());
        T.sscls.insert(T.sscls.end(), ssc.begin(), ssc.end());
        T.sswords.insert(T.sswords.end(), ssw.begin(), ssw.end());
        T.sslos.insert(T.sslos.end(), ssl.begin(), ssl.end());
        T.zs.insert(T.zs.end(), z.begin(), z.end());
        T.cs.insert(T.cs.end(), c.begin(), c.end());
        T.state_amps += 2ull << n;
        T.tabs += tab;
        T.tickets += e.W;
        T.parts += (int64_t)e.W * e.K + e.W;
        if (T.zs.size() > (size_t)INT32_MAX || T.tickets > INT32_MAX || T.parts > INT32_MAX ||
            T.lruns.size() > (size_t)INT32_MAX || T.tabs > INT32_MAX || T.sslos.size() > (size_t)INT32_MAX)
            raise(QF_E_ARG, "batch too large");
    }
    B.nentries = (int)T.ent.size();
    B.entry_out.clear();
    for (const BatchEntry &e : T.ent)
        B.entry_out.push_back(e.out);
    B.status.assign((size_t)count, QF_OK);
    B.total_tickets = (unsigned)T.tickets;
    B.grid = std::min<unsigned>(B.grid, B.total_tickets);
    B.state_bytes = T.state_amps * sizeof(double2);
}

// Device layout: one contiguous region, every array 256-byte aligned.
struct Layout {
    size_t off[22];
    size_t total;
};

Layout batch_layout(const qf_batch &B, const BatchHost &T)
{
    const size_t sizes[22] = {
        T.ent.size() * sizeof(BatchEntry), std::max<size_t>(T.runs.size(), 1) * sizeof(RunDesc),
        T.groups.size() * sizeof(GroupDesc), T.zs.size() * sizeof(uint32_t), T.cs.size() * sizeof(double),
        (size_t)std::max<int64_t>(B.K_total, 1) * sizeof(double), B.state_bytes,
        (size_t)T.parts * sizeof(double), T.ent.size() * kSyncWords * sizeof(unsigned), sizeof(unsigned),
        T.ent.size() * sizeof(unsigned),
        (size_t)B.count * sizeof(double), (size_t)std::max<int64_t>(B.K_total, 1) * sizeof(double),
        std::max<size_t>(T.segs.size(), 1) * sizeof(Segment), std::max<size_t>(T.lruns.size(), 1) * sizeof(LocalRun),
        std::max<size_t>(T.sscls.size(), 1) * sizeof(SsCls), (size_t)std::max<int64_t>(T.tabs, 1) * sizeof(double2),
        std::max<size_t>(T.sswords.size(), 1) * sizeof(uint32_t), std::max<size_t>(T.sslos.size(), 1) * sizeof(SsLo),
        std::max<size_t>(T.lruns.size(), 1) * sizeof(ApplyTriple), std::max<size_t>(T.lruns.size(), 1) * sizeof(AdjPair),
        T.smap.size() * sizeof(uint32_t)};
    Layout L;
    size_t at = 0;
    for (int i = 0; i < 22; i++) {
        L.off[i] = at;
        at += (sizes[i] + 255) & ~(size_t)255;
    }
    L.total = at;
    return L;
}

void batch_bind(qf_batch &B, char *base, const Layout &L)
{
    B.d_entries = (BatchEntry *)(base + L.off[0]);
    B.d_runs = (RunDesc *)(base + L.off[1]);
    B.d_groups = (GroupDesc *)(base + L.off[2]);
    B.d_z = (uint32_t *)(base + L.off[3]);
    B.d_c = (double *)(base + L.off[4]);
    B.d_theta = (double *)(base + L.off[5]);
    B.d_states = (double2 *)(base + L.off[6]);
    B.d_partials = (double *)(base + L.off[7]);
    B.d_sync = (unsigned *)(base + L.off[8]);
    B.d_ticket = (unsigned *)(base + L.off[9]);
    B.d_err = (unsigned *)(base + L.off[10]);
    B.d_E = (double *)(base + L.off[11]);
    B.d_grad = (double *)(base + L.off[12]);
    B.d_segs = (Segment *)(base + L.off[13]);
    B.d_lruns = (LocalRun *)(base + L.off[14]);
    B.d_sscls = (SsCls *)(base + L.off[15]);
    B.d_tabs = (double2 *)(base + L.off[16]);
    B.d_sswords = (uint32_t *)(base + L.off[17]);
    B.d_sslos = (SsLo *)(base + L.off[18]);
    B.d_atrip = (ApplyTriple *)(base + L.off[19]);
    B.d_apairs = (AdjPair *)(base + L.off[20]);
    B.d_smap = (uint32_t *)(base + L.off[21]);
}

__global__ void k_fill_zero(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void batch_upload(qf_batch &B, const BatchHost &T, hipStream_t s)
{
    QF_HIP(hipMemcpyAsync(B.d_entries, T.ent.data(), T.ent.size() * sizeof(BatchEntry), hipMemcpyHostToDevice, s));
    if (!T.runs.empty())
        QF_HIP(hipMemcpyAsync(B.d_runs, T.runs.data(), T.runs.size() * sizeof(RunDesc), hipMemcpyHostToDevice, s));
    if (!T.segs.empty())
        QF_HIP(hipMemcpyAsync(B.d_segs, T.segs.data(), T.segs.size() * sizeof(Segment), hipMemcpyHostToDevice, s));
    if (!T.lruns.empty()) {
        QF_HIP(hipMemcpyAsync(B.d_lruns, T.lruns.data(), T.lruns.size() * sizeof(LocalRun), hipMemcpyHostToDevice,
                              s));
        QF_HIP(hipMemcpyAsync(B.d_atrip, T.atrip.data(), T.atrip.size() * sizeof(ApplyTriple), hipMemcpyHostToDevice,
                              s));
        QF_HIP(hipMemcpyAsync(B.d_apairs, T.apairs.data(), T.apairs.size() * sizeof(AdjPair), hipMemcpyHostToDevice,
                              s));
    }
    QF_HIP(hipMemcpyAsync(B.d_smap, T.smap.data(), T.smap.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    QF_HIP(hipMemcpyAsync(B.d_groups, T.groups.data(), T.groups.size() * sizeof(GroupDesc), hipMemcpyHostToDevice,
                          s));
    if (!T.sscls.empty()) {
        QF_HIP(hipMemcpyAsync(B.d_sscls, T.sscls.data(), T.sscls.size() * sizeof(SsCls), hipMemcpyHostToDevice, s));
        QF_HIP(hipMemcpyAsync(B.d_sswords, T.sswords.data(), T.sswords.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
        QF_HIP(hipMemcpyAsync(B.d_sslos, T.sslos.data(), T.sslos.size() * sizeof(SsLo), hipMemcpyHostToDevice, s));
    }
    QF_HIP(hipMemcpyAsync(B.d_z, T.zs.data(), T.zs.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    QF_HIP(hipMemcpyAsync(B.d_c, T.cs.data(), T.cs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    const int64_t ng = std::max<int64_t>(B.K_total, 1);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(1024, (ng + 255) / 256)), dim3(256), 0, s,
                       B.d_grad, ng);
    QF_HIP(hipGetLastError());
    QF_HIP(hipStreamSynchronize(s));  // the host tables are freed on return
}

void batch_kernels(qf_batch &B, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(std::max(1, std::min(64, (B.nentries * kSyncWords + 255) / 256))), dim3(256), 0, s,
                       B.d_sync, B.nentries, B.d_ticket, B.d_err);
    hipLaunchKernelGGL(k_batch, dim3(B.grid), dim3(kBT), 0, s, B.d_entries, B.nentries, B.total_tickets,
                       B.d_runs, B.d_segs, B.d_lruns, B.d_atrip, B.d_apairs, B.d_smap, B.d_groups, B.d_sscls, B.d_sswords, B.d_sslos, B.d_tabs, B.d_z, B.d_c, B.d_theta, B.d_states, B.d_partials, B.d_sync,
                       B.d_ticket, B.d_err, B.d_E, B.d_grad, B.spin_limit, B.mb_E, B.mb_grad, B.mb_flag);
    QF_HIP(hipGetLastError());
}

// owned mode, graph-capturable: pinned theta -> device, kernels, results -> pinned
void batch_enqueue(qf_batch &B, hipStream_t s)
{
    QF_HIP(hipMemcpyAsync(B.d_theta, B.h_theta, (size_t)std::max<int64_t>(B.K_total, 1) * sizeof(double),
                          hipMemcpyHostToDevice, s));
    batch_kernels(B, s);
    QF_HIP(hipMemcpyAsync(B.h_E, B.d_E, (size_t)B.count * sizeof(double), hipMemcpyDeviceToHost, s));
    QF_HIP(hipMemcpyAsync(B.h_grad, B.d_grad, (size_t)std::max<int64_t>(B.K_total, 1) * sizeof(double),
                          hipMemcpyDeviceToHost, s));
}

// Per-instance status of the last launch (caller order); QF_E_HIP if any
// instance's team barrier timed out.
int check_err(qf_batch &B)
{
    std::vector<unsigned> err((size_t)B.nentries, 0u);
    QF_HIP(hipMemcpy(err.data(), B.d_err, err.size() * sizeof(unsigned), hipMemcpyDeviceToHost));
    B.status.assign((size_t)B.count, QF_OK);
    int bad = 0;
    for (int e = 0; e < B.nentries; e++)
        if (err[(size_t)e]) {
            B.status[(size_t)B.entry_out[(size_t)e]] = QF_E_HIP;
            bad++;
        }
    if (bad)
        return fail(QF_E_HIP, "qf_batch: %d of %d instances failed, a team barrier timed out (spin limit %u polls)",
                    bad, B.count, B.spin_limit);
    return QF_OK;
}

} // namespace qf

using namespace qf;

extern "C" int qf_batch_create(int count, const int *n_qubits, const uint64_t *occ_mask, const qf_term *const *A,
                               const int64_t *K, const qf_term *const *H, const int64_t *const *group_off,
                               const int64_t *n_groups, const int *team, qf_batch **out)
{
    return guarded([&]() -> int {
        if (!out)
            return fail(QF_E_ARG, "qf_batch_create: out is NULL");
        *out = nullptr;
        qf_batch *B = new qf_batch();
        try {
            BatchHost T;
            batch_assemble(*B, T, count, n_qubits, occ_mask, A, K, H, group_off, n_groups, team);
            const Layout L = batch_layout(*B, T);
            char *base = dev_alloc<char>(L.total);
            B->owns_device = true;
            B->d_base = base;
            batch_bind(*B, base, L);
            B->device_bytes = L.total;
            batch_upload(*B, T, nullptr);
            const size_t nk = (size_t)std::max<int64_t>(B->K_total, 1);
            QF_HIP(hipHostMalloc((void **)&B->h_theta, nk * sizeof(double), hipHostMallocDefault));
            QF_HIP(hipHostMalloc((void **)&B->h_grad, nk * sizeof(double), hipHostMallocDefault));
            QF_HIP(hipHostMalloc((void **)&B->h_E, (size_t)B->count * sizeof(double), hipHostMallocDefault));
            QF_HIP(hipEventCreateWithFlags(&B->done, hipEventDisableTiming));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
        return QF_OK;
    });
}

extern "C" int qf_batch_create_arena(int count, const int *n_qubits, const uint64_t *occ_mask,
                                     const qf_term *const *A, const int64_t *K, const qf_term *const *H,
                                     const int64_t *const *group_off, const int64_t *n_groups, const int *team,
                                     int concurrent, void *arena, int64_t arena_bytes, int64_t *need_bytes,
                                     void *stream, qf_batch **out)
{
    return guarded([&]() -> int {
        if (out)
            *out = nullptr;
        if (concurrent < 1)
            return fail(QF_E_ARG, "qf_batch_create_arena: concurrent < 1");
        qf_batch *B = new qf_batch();
        try {
            BatchHost T;
            batch_assemble(*B, T, count, n_qubits, occ_mask, A, K, H, group_off, n_groups, team, concurrent);
            const Layout L = batch_layout(*B, T);
            if (need_bytes)
                *need_bytes = (int64_t)L.total;
            if (!arena) {
                delete B;
                return QF_OK;
            }
            if (!out)
                raise(QF_E_ARG, "qf_batch_create_arena: out is NULL");
            if ((uintptr_t)arena % 256)
                raise(QF_E_ARG, "qf_batch_create_arena: arena must be 256-byte aligned");
            if (arena_bytes < (int64_t)L.total)
                raise(QF_E_SIZE, "qf_batch_create_arena: arena of " + std::to_string(arena_bytes) +
                                     " bytes, need " + std::to_string(L.total));
            B->owns_device = false;
            batch_bind(*B, (char *)arena, L);
            B->device_bytes = L.total;
            batch_upload(*B, T, (hipStream_t)stream);
            QF_HIP(hipEventCreateWithFlags(&B->done, hipEventDisableTiming));
        } catch (...) {
            delete B;
            throw;
        }
        *out = B;
        return QF_OK;
    });
}

extern "C" int qf_batch_teams(int count, const int *n_qubits, const int64_t *K, const int64_t *n_strings,
                              const int *team, int grid, int concurrent, int *W_out)
{
    return guarded([&]() -> int {
        if (count < 1 || !n_qubits || !K || !n_strings || !W_out || grid < 1 || concurrent < 1)
            return fail(QF_E_ARG, "qf_batch_teams: bad arguments");
        for (int i = 0; i < count; i++)
            if (n_qubits[i] < 1 || n_qubits[i] > 30 || K[i] < 0 || n_strings[i] < 0)
                return fail(QF_E_RANGE, "qf_batch_teams: instance %d out of range", i);
        team_sizes(count, n_qubits, K, n_strings, team, (unsigned)grid, concurrent, W_out);
        return QF_OK;
    });
}

extern "C" int qf_batch_resident_grid(int *grid)
{
    return guarded([&]() -> int {
        if (!grid)
            return fail(QF_E_ARG, "qf_batch_resident_grid: grid is NULL");
        *grid = (int)resident_grid();
        return QF_OK;
    });
}

extern "C" int qf_batch_status(const qf_batch *b, int *status)
{
    if (!b || !status)
        return fail(QF_E_ARG, "qf_batch_status: null argument");
    for (int i = 0; i < b->count; i++)
        status[i] = b->status[(size_t)i];
    return QF_OK;
}

extern "C" int qf_batch_destroy(qf_batch *b)
{
    delete b;
    return QF_OK;
}

extern "C" int qf_batch_info(const qf_batch *b, int *team, int64_t *state_bytes, int *grid)
{
    if (!b)
        return fail(QF_E_ARG, "qf_batch_info: batch is NULL");
    if (team)
        for (int i = 0; i < b->count; i++)
            team[i] = b->W[(size_t)i];
    if (state_bytes)
        *state_bytes = (int64_t)b->state_bytes;
    if (grid)
        *grid = (int)b->grid;
    return QF_OK;
}

extern "C" int qf_batch_set_spin_limit(qf_batch *b, uint32_t polls)
{
    if (!b || polls == 0)
        return fail(QF_E_ARG, "qf_batch_set_spin_limit: bad arguments");
    b->spin_limit = polls;
    b->drop_graph();  // a captured launch holds the old limit
    return QF_OK;
}

extern "C" int qf_mailbox_alloc(int64_t bytes, void **out)
{
    return guarded([&]() -> int {
        if (!out || bytes <= 0)
            return fail(QF_E_ARG, "qf_mailbox_alloc: bad arguments");
        *out = nullptr;
        void *p = nullptr;
        const hipError_t e = hipHostMalloc(&p, (size_t)bytes, hipHostMallocCoherent | hipHostMallocMapped);
        if (e != hipSuccess)
            return fail(QF_E_NOMEM, "qf_mailbox_alloc: %s", hipGetErrorString(e));
        std::memset(p, 0, (size_t)bytes);
        *out = p;
        return QF_OK;
    });
}

extern "C" int qf_mailbox_free(void *p)
{
    if (p)
        (void)hipHostFree(p);
    return QF_OK;
}

extern "C" int qf_batch_mailbox_bytes(const qf_batch *B, int64_t *bytes)
{
    if (!B || !bytes)
        return fail(QF_E_ARG, "qf_batch_mailbox_bytes: null argument");
    *bytes = 8 * (int64_t)B->count + 8 * B->K_total + 4 * (int64_t)B->count;
    return QF_OK;
}

extern "C" int qf_batch_launch_mailbox(qf_batch *B, const double *theta, void *mailbox, int64_t mailbox_bytes,
                                       void *stream)
{
    return guarded([&]() -> int {
        if (!B)
            return fail(QF_E_ARG, "qf_batch_launch_mailbox: batch is NULL");
        int64_t need = 0;
        qf_batch_mailbox_bytes(B, &need);
        if (!mailbox || mailbox_bytes < need)
            return fail(QF_E_SIZE, "qf_batch_launch_mailbox: mailbox of %lld bytes, need %lld",
                        (long long)mailbox_bytes, (long long)need);
        char *m = (char *)mailbox;
        B->mb_E = (double *)m;
        B->mb_grad = (double *)(m + 8 * (size_t)B->count);
        B->mb_flag = (unsigned *)(m + 8 * (size_t)B->count + 8 * (size_t)B->K_total);
        std::memset(B->mb_flag, 0, 4 * (size_t)B->count);
        const int st = qf_batch_launch(B, theta, stream);
        B->mb_E = nullptr;
        B->mb_grad = nullptr;
        B->mb_flag = nullptr;
        return st;
    });
}

extern "C" int qf_batch_launch(qf_batch *B, const double *theta, void *stream)
{
    return guarded([&]() -> int {
        if (!B || (B->K_total > 0 && !theta))
            return fail(QF_E_ARG, "qf_batch_launch: null argument");
        hipStream_t s = (hipStream_t)stream;
        const size_t nk = (size_t)std::max<int64_t>(B->K_total, 1);
        B->theta_host.assign(nk, 0.0);
        if (B->K_total > 0)
            std::memcpy(B->theta_host.data(), theta, (size_t)B->K_total * sizeof(double));
        QF_HIP(hipMemcpyAsync(B->d_theta, B->theta_host.data(), nk * sizeof(double), hipMemcpyHostToDevice, s));
        batch_kernels(*B, s);
        QF_HIP(hipEventRecord(B->done, s));
        B->launched = true;
        return QF_OK;
    });
}

extern "C" int qf_batch_poll(qf_batch *B)
{
    if (!B || !B->launched)
        return fail(QF_E_ARG, "qf_batch_poll: nothing launched");
    const hipError_t e = hipEventQuery(B->done);
    if (e == hipSuccess)
        return QF_OK;
    if (e == hipErrorNotReady)
        return 1;
    return fail(QF_E_HIP, "qf_batch_poll: %s", hipGetErrorString(e));
}

extern "C" int qf_batch_collect(qf_batch *B, double *E_out, double *dE_dtheta)
{
    return guarded([&]() -> int {
        if (!B || !B->launched || !E_out)
            return fail(QF_E_ARG, "qf_batch_collect: nothing launched or E_out is NULL");
        QF_HIP(hipEventSynchronize(B->done));
        B->launched = false;
        QF_HIP(hipMemcpy(E_out, B->d_E, (size_t)B->count * sizeof(double), hipMemcpyDeviceToHost));
        if (dE_dtheta && B->K_total > 0)
            QF_HIP(hipMemcpy(dE_dtheta, B->d_grad, (size_t)B->K_total * sizeof(double), hipMemcpyDeviceToHost));
        return check_err(*B);
    });
}

extern "C" int qf_batch_run(qf_batch *B, const double *theta, double *E_out, double *dE_dtheta, int use_graph,
                            void *stream)
{
    return guarded([&]() -> int {
        if (!B || !E_out || (B->K_total > 0 && !theta))
            return fail(QF_E_ARG, "qf_batch_run: null argument");
        if (!B->owns_device) {
            int st = qf_batch_launch(B, theta, stream);
            return st != QF_OK ? st : qf_batch_collect(B, E_out, dE_dtheta);
        }
        hipStream_t s = (hipStream_t)stream;
        if (B->K_total > 0)
            std::memcpy(B->h_theta, theta, (size_t)B->K_total * sizeof(double));
        if (use_graph) {
            if (B->exec && B->graph_stream != s)
                B->drop_graph();
            if (!B->exec) {
                hipStream_t cs = s;
                bool own = false;
                if (!cs) {  // the legacy default stream cannot be captured
                    QF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                    own = true;
                }
                QF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                try {
                    batch_enqueue(*B, cs);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(cs, &g);
                    if (g)
                        (void)hipGraphDestroy(g);
                    if (own)
                        (void)hipStreamDestroy(cs);
                    throw;
                }
                QF_HIP(hipStreamEndCapture(cs, &B->graph));
                if (own)
                    QF_HIP(hipStreamDestroy(cs));
                QF_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
                B->graph_stream = s;
            }
            QF_HIP(hipGraphLaunch(B->exec, s));
        } else {
            batch_enqueue(*B, s);
        }
        QF_HIP(hipStreamSynchronize(s));
        std::memcpy(E_out, B->h_E, (size_t)B->count * sizeof(double));
        if (dE_dtheta && B->K_total > 0)
            std::memcpy(dE_dtheta, B->h_grad, (size_t)B->K_total * sizeof(double));
        return check_err(*B);
    });
}
