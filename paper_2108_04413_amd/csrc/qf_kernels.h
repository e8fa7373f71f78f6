// Device-side types and helpers shared by the plain kernels (qf_device.hip)
// and the persistent batched kernel (qf_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qf {

constexpr int kBlock = 256;
constexpr int kItems = 4;        // amplitude pairs per thread per step
constexpr int kMaxRun = 8;       // strings per fused run
constexpr int kMaxRank = 6;      // rank of a run's sign patterns (table <= 64)
constexpr int kMaxBlocks = 2048; // cap of grid-stride launches (8 blocks / CU)

struct RunDesc {
    uint32_t x, z0, hbit, a0;
    uint32_t b[kMaxRank];
    int32_t r, k0, m, tab;
    uint8_t e[kMaxRun];
    int8_t s[kMaxRun];
};

struct GroupDesc {
    uint32_t x, hbit;
    int32_t k0, kre, k1;  // [k0,kre): real phase, [kre,k1): imaginary phase
    // item-sign pattern of the sigma passes (items 512 apart): bits 0-3 the
    // value of (z >> kPatBit) & 3 shared by all real-phase strings, bits 4-7
    // that of the imaginary-phase strings, 0xF where the strings differ
    int32_t pat;
};
constexpr int kPatBit = 9;

// Blocked application of consecutive runs.  A segment is a range of runs
// whose flip masks all lie inside a set Q of B qubits that contains the
// lowest q0 qubits; the state splits into 2^(n-B) sub-cubes (fixed values of
// the other qubits), each loaded into LDS once, updated by every run of the
// segment, and written back.  Masks of a run are given both in the full
// index space (for the sub-cube's fixed bits) and compressed to Q (pext).
constexpr int kSegTab = 512;  // (cos, sin) entries of one segment, staged in LDS
constexpr int kSegStr = 512;  // strings of one segment (blocked adjoint accumulators in LDS)

struct Segment {
    uint32_t Q;      // qubits of the sub-cube
    int32_t q0;      // Q contains qubits 0 .. q0-1 (q0 >= min(6, B))
    int32_t r0, r1;  // runs [r0, r1) of the segment (LocalRun array)
    uint32_t hi[8];  // positions of Q's qubits above q0, ascending
    int32_t nhi;
    int32_t tab0, ntab;  // the segment's runs use tab[tab0, tab0 + ntab)
    int32_t pad;
};

// Sub-cube kernels give thread t the items t + k * kItemStride (k = 0, 1,
// ...) of a run: pair index j for a flip run, amplitude index y for a
// diagonal one.  Both the table index u(y) and the Z-parity par(y & z0) are
// affine in y and the item offsets are the same for every thread, so their
// parts from item k's offset are tabulated per run (LocalRun::itm, byte k):
//   flip run:     y_k = insert0(k * kItemStride, hbit),
//                 byte k = u(y_k) | par(y_k & z0) << 6,  k < 4;
//   diagonal run: byte k = u(k * kItemStride),            k < 8.
// Every kernel that has more than one item per thread runs kItemStride threads.
constexpr int kItemStride = 512;
constexpr int kSegRuns = kSegStr;  // runs of one segment (each has >= 1 string)

struct LocalRun {
    uint32_t x, hbit, z0, a0;       // local flip mask, its highest bit, local z0, i^a0
    uint32_t b[kMaxRank];           // local GF(2) basis masks (zero beyond the rank)
    uint32_t z0f;                   // full-space z0
    uint32_t bf[kMaxRank];          // full-space basis masks
    int32_t r, tab;
    int32_t k0, m;                  // the run's strings (as in RunDesc)
    uint8_t e[kMaxRun];
    int8_t s[kMaxRun];
    uint32_t itm[2];                // per-item table-index and parity parts
};
static_assert(kMaxRun == 8, "e and s of a LocalRun fill one 64-bit word each");

// Tiled energy, merged form.  Inside a tile pair the bits of y above the tile
// are fixed, so the factor (-1)^popcount(y_hi & z_hi) of every string is a
// per-item constant: strings of a group that share (phase, z_lo) merge into
// one "lo-term" whose coefficient is summed per work item.  A group's strings
// are records sorted by (phase, z_lo); the last record of each lo-term has
// `emit` set.
struct ERec {
    uint32_t zlo;   // z & (2^L - 1)
    uint32_t emit;  // 1 on the last string of a lo-term
    uint32_t zhi;   // z >> L, as a tile-index mask
    uint32_t pad;
    double c;       // coefficient with the sign of i^popcount(x&z) folded in
    double pad2;
};

// Groups whose flip masks share the bits above the tile (x >> L == xh):
// one tiled energy pass covers all of them.
struct ClassDesc {
    uint32_t xh;     // flip bits above the tile, as a tile-index mask
    uint32_t hb;     // highest set bit of xh (0 if xh == 0)
    int32_t g0, g1;  // group range
};

// Streaming energy: the work order interleaves the classes.  Each class is cut
// into pieces of 2^(n-L-1) tile pairs (the class with no flip bits above the
// tile has 2^(n-L) tiles and so two pieces); a round visits every piece once,
// at the same tile-pair offset, so ALU-heavy classes are spread over the whole
// launch instead of running back to back.
struct VClass {
    uint32_t xh, hb;  // as in ClassDesc
    uint32_t j0;      // first tile-pair index of the piece
    int32_t g0, g1;   // groups of the class
    int32_t r0, r1;   // records of the class (merged form)
    uint32_t pad;
};

// ------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t insert0(uint32_t j, uint32_t bit)
{
    const uint32_t lo = j & ((1u << bit) - 1u);
    return ((j ^ lo) << 1) | lo;
}

// Sub-cube sc of a segment: its index bits, in order, at the qubits outside
// Q (Q = qubits 0..q0-1 and hi[0] < ... < hi[nhi-1]): shift past the low
// run, then open a zero at each of Q's higher qubits, lowest first.
__device__ __forceinline__ uint32_t subcube_base(uint32_t sc, const Segment &sg)
{
    uint32_t v = sc << sg.q0;
#pragma unroll
    for (int j = 0; j < 8; j++)
        if (j < sg.nhi)
            v = insert0(v, sg.hi[j]);
    return v;
}

__device__ __forceinline__ uint32_t par(uint32_t v) { return __popc(v) & 1u; }

// v * i^k
__device__ __forceinline__ double2 mul_ik(uint32_t k, double2 v)
{
    double re = (k & 1u) ? -v.y : v.x;
    double im = (k & 1u) ? v.x : v.y;
    if (k & 2u) {
        re = -re;
        im = -im;
    }
    return make_double2(re, im);
}

__device__ __forceinline__ double flip(double v, uint32_t p)
{
    // multiply by (-1)^p on the sign bit
    return __hiloint2double(__double2hiint(v) ^ (int)(p << 31), __double2loint(v));
}

// v with its sign bit xor-ed with bit 31 of m
__device__ __forceinline__ double flip31(double v, uint32_t m)
{
    return __hiloint2double(__double2hiint(v) ^ (int)m, __double2loint(v));
}

// A run's item table as one 64-bit word, and its byte k.  (Shifts, not an
// index: a run-time index into a register copy of the descriptor would put
// the copy in scratch memory.)
__device__ __forceinline__ uint64_t item_table(const LocalRun &d)
{
    return (uint64_t)d.itm[0] | ((uint64_t)d.itm[1] << 32);
}

__device__ __forceinline__ uint32_t item_part(uint64_t it, int k)
{
    return (uint32_t)(it >> (8 * k)) & 0xffu;
}

// Rotation of a pair by the exponential of a run.  Writing the phase of the
// partner amplitude as i^a0 (-1)^p, with a0 fixed by the run and p the
// Z-parity of the partner, both exp(-i theta P) and exp(+i theta P) take
// (a, b) = (psi[y1], psi[y1 ^ x]) to
//   a' = c a + s2 i^w b,    b' = c b + s1 i^w a
// with w = 0 or 1 (SWAP) and s1, s2 = +-s: the rest of the phase, the
// direction and the two parities are all signs.  i v = (-v.y, v.x).
template <bool SWAP> __device__ __forceinline__ void rot_pair(double c, double s1, double s2, double2 &a, double2 &b)
{
    const double2 a0 = a, b0 = b;
    if (SWAP) {
        a = make_double2(c * a0.x - s2 * b0.y, c * a0.y + s2 * b0.x);
        b = make_double2(c * b0.x - s1 * a0.y, c * b0.y + s1 * a0.x);
    } else {
        a = make_double2(c * a0.x + s2 * b0.x, c * a0.y + s2 * b0.y);
        b = make_double2(c * b0.x + s1 * a0.x, c * b0.y + s1 * a0.y);
    }
}

// Fixed-bit parities of every run of a segment for one sub-cube:
// pbz[r] = sum_q par(base & bf_q) << q | par(base & z0f) << 6.
__device__ __forceinline__ void sub_parities(const LocalRun *__restrict__ lr, int r0, int nr, uint32_t base,
                                             uint32_t *pbz, int tid, int nt)
{
    for (int r = tid; r < nr; r += nt) {
        const LocalRun &d = lr[r0 + r];
        uint32_t v = par(base & d.z0f) << 6;
#pragma unroll
        for (int q = 0; q < kMaxRank; q++)
            v |= par(base & d.bf[q]) << q;
        pbz[r] = v;
    }
}

// Wavefront sums of 8 values per lane with 10 exchanges instead of 48, all
// of them register moves (DPP and the gfx950 lane swaps), none through the
// LDS crossbar.  Three halving steps over lane bits 0, 1 and 4 (each lane
// keeps half of its values and receives the other half from its partner)
// leave lane l with value sum8_index(l) = 4 b0 + 2 b1 + b4 summed over the 8
// lanes that share bits 2, 3 and 5; two rotations within each 16-lane row
// add the lanes that differ in bits 2 and 3 (the rotation's direction does
// not matter: ror 4 then ror 8 visits all four), and a swap of the two
// 32-lane halves adds bit 5.  Lanes with bits 2, 3 and 5 clear
// (sum8_writer) hold the 8 totals.  The order of additions is fixed.
__device__ __forceinline__ int sum8_index(int lane)
{
    return 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 4) & 1);
}

__device__ __forceinline__ bool sum8_writer(int lane) { return (lane & 0x2c) == 0; }

// Every control used here (quad_perm, row_ror with all rows and banks
// enabled) reads a lane inside the same row, so no lane falls back to the
// old value and none needs to be supplied (bound_ctrl).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xb1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4e;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRor4 = 0x124; // row_ror:4
constexpr int kDppRor8 = 0x128; // row_ror:8

// the value of lane l ^ 16 (lanes exchange 16-lane rows 0 <-> 1, 2 <-> 3)
__device__ __forceinline__ double xor16_f64(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    // one result of each swap is this lane's own word, the other the
    // partner's; where both are equal either is right
    const bool first_is_own = (int)pl[0] == lo && (int)ph[0] == hi;
    return __hiloint2double(first_is_own ? (int)ph[1] : (int)ph[0], first_is_own ? (int)pl[1] : (int)pl[0]);
}

// v(l) + v(l ^ 32): the swap leaves each lane one word of each half
__device__ __forceinline__ double sum_xor32_f64(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)ph[0], (int)pl[0]) + __hiloint2double((int)ph[1], (int)pl[1]);
}

__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane)
{
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b4 = (lane >> 4) & 1;
    double h4[4], h2[2];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const double send = b0 ? v[k] : v[k + 4];
        const double keep = b0 ? v[k + 4] : v[k];
        h4[k] = keep + dpp_f64<kDppXor1>(send);
    }
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const double send = b1 ? h4[k] : h4[k + 2];
        const double keep = b1 ? h4[k + 2] : h4[k];
        h2[k] = keep + dpp_f64<kDppXor2>(send);
    }
    double h;
    {
        const double send = b4 ? h2[0] : h2[1];
        const double keep = b4 ? h2[1] : h2[0];
        h = keep + xor16_f64(send);
    }
    h += dpp_f64<kDppRor4>(h);
    h += dpp_f64<kDppRor8>(h);
    return sum_xor32_f64(h);
}

// One thread's share of one run in the 8 Walsh sums
// W[e] += sum_k (-1)^popcount(u_k & e) q_k over its items k, whose table
// indices are u_k = u0 ^ du[k] with du[k] the same for every thread:
// W[e] += (-1)^popcount(u0 & e) sum_k (-1)^popcount(du[k] & e) q_k, the
// inner signs uniform (FMAs by +-1.0) and the outer one a sign flip.  Equal
// bit for bit to adding the signed terms one at a time (negation commutes
// with rounding; an FMA by +-1.0 rounds as the add it stands for).
__device__ __forceinline__ double pm_one(uint32_t m31);
template <int N>
__device__ __forceinline__ void walsh_add(double (&acc)[kMaxRun], uint32_t u0, const uint32_t (&du)[N],
                                          const double (&q)[N])
{
    const uint32_t b1 = u0 << 31, b2 = (u0 >> 1) << 31, b4 = (u0 >> 2) << 31;
    const uint32_t sb[kMaxRun] = {0u, b1, b2, b1 ^ b2, b4, b1 ^ b4, b2 ^ b4, b1 ^ b2 ^ b4};
    // the uniform signs (-1)^popcount(du[k] & e) by the same XOR table
    uint32_t sd[N][kMaxRun];
#pragma unroll
    for (int k = 1; k < N; k++) {
        const uint32_t c1 = du[k] << 31, c2 = (du[k] >> 1) << 31, c4 = (du[k] >> 2) << 31;
        const uint32_t t[kMaxRun] = {0u, c1, c2, c1 ^ c2, c4, c1 ^ c4, c2 ^ c4, c1 ^ c2 ^ c4};
#pragma unroll
        for (int e = 0; e < kMaxRun; e++)
            sd[k][e] = t[e];
    }
#pragma unroll
    for (int e = 0; e < kMaxRun; e++) {
        double r = q[0];
#pragma unroll
        for (int k = 1; k < N; k++)
            r = fma(pm_one(sd[k][e]), q[k], r);
        acc[e] += flip31(r, sb[e]);
    }
}

// GF(2) coordinates of y against the masks bm (zero beyond the run's
// rank r): bit q is the parity of y & bm[q].  Linear in y.  Runs of rank
// <= 3 (every single and double excitation) skip the upper three masks on a
// uniform branch.
__device__ __forceinline__ uint32_t gf2_coords(uint32_t y, const uint32_t (&bm)[kMaxRank], int r)
{
    uint32_t u = par(y & bm[0]) | (par(y & bm[1]) << 1) | (par(y & bm[2]) << 2);
    if (r > 3) {
#pragma unroll
        for (int q = 3; q < kMaxRank; q++)
            u ^= par(y & bm[q]) << q;
    }
    return u;
}

__device__ __forceinline__ uint32_t run_coords(const RunDesc &d, uint32_t y)
{
    // Unrolled to the maximum rank so that every index is a constant: a
    // descriptor copied out of global memory then stays in registers.
    uint32_t u = 0;
#pragma unroll
    for (int q = 0; q < kMaxRank; q++)
        if (q < d.r)
            u |= par(y & d.b[q]) << q;
    return u;
}

// D_g(y_i) = sum_{k in g} c_k omega_k(y_i) for kItems indices at once; every
// string is loaded once (scalar) and applied to all items.
__device__ __forceinline__ void group_d(const GroupDesc &g, const uint32_t *__restrict__ zs,
                                        const double *__restrict__ cs, const uint32_t (&y)[kItems],
                                        double (&dre)[kItems], double (&dim)[kItems])
{
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        dre[i] = 0.0;
        dim[i] = 0.0;
    }
#pragma unroll 2
    for (int k = g.k0; k < g.kre; k++) {
        const uint32_t z = zs[k];
        const double c = cs[k];
#pragma unroll
        for (int i = 0; i < kItems; i++)
            dre[i] += flip(c, par(y[i] & z));
    }
    for (int k = g.kre; k < g.k1; k++) {
        const uint32_t z = zs[k];
        const double c = cs[k];
#pragma unroll
        for (int i = 0; i < kItems; i++)
            dim[i] += flip(c, par(y[i] & z));
    }
}

// D_g at the four indices Y ^ (i << LS), i = 0..3, for the sigma passes,
// whose items are 2^LS apart with bits LS and LS + 1 of the first item
// clear.  String k's sign at item i is (-1)^popcount(Y & z_k) times
// (-1)^(i0 z_k[LS] + i1 z_k[LS + 1]); the first factor is computed once per
// thread, the second is the same for the whole wavefront and enters as an
// FMA by +-1.0 (exact, so equal to the signed add).  (A host table of the
// item signs, 32 B per string, was slower in the batched kernel: many
// instances' tables thrash the scalar cache.)
__device__ __forceinline__ double pm_one(uint32_t m31)
{
    return __hiloint2double((int)(0x3ff00000u ^ m31), 0);
}

template <int LS>
__device__ __forceinline__ void group_d4_part(int k0, int k1, const uint32_t *__restrict__ zs,
                                              const double *__restrict__ cs, uint32_t Y, double (&d)[4])
{
#pragma unroll 2
    for (int k = k0; k < k1; k++) {
        // both loads first: they then share one wait (loading c after the
        // sign arithmetic on z had the compiler wait for each separately)
        const uint32_t z = zs[k];
        const double c = cs[k];
        const uint32_t m1 = (z >> LS) << 31, m2 = (z >> (LS + 1)) << 31;
        const double t = flip31(c, (uint32_t)__popc(Y & z) << 31);
        d[0] += t;
        d[1] = fma(pm_one(m1), t, d[1]);
        d[2] = fma(pm_one(m2), t, d[2]);
        d[3] = fma(pm_one(m1 ^ m2), t, d[3]);
    }
}

// As group_d4_part for LS = kPatBit, with the strings' common item-sign
// pattern p (0..3) when they share one: then the signed sum runs once and
// item i takes (-1)^popcount(i & p) times it (bit for bit the per-item sums:
// the item signs are exact); p > 3 falls back to per-string signs.
__device__ __forceinline__ void group_d4_part_pat(int k0, int k1, int p, const uint32_t *__restrict__ zs,
                                                  const double *__restrict__ cs, uint32_t Y, double (&d)[4])
{
    if (p > 3) {
        group_d4_part<kPatBit>(k0, k1, zs, cs, Y, d);
        return;
    }
    double a = -0.0;
#pragma unroll 2
    for (int k = k0; k < k1; k++) {
        const uint32_t z = zs[k];
        const double c = cs[k];
        a += flip31(c, (uint32_t)__popc(Y & z) << 31);
    }
    const uint32_t m1 = (uint32_t)p << 31, m2 = ((uint32_t)p >> 1) << 31;
    d[0] += a;
    d[1] += flip31(a, m1);
    d[2] += flip31(a, m2);
    d[3] += flip31(a, m1 ^ m2);
}

template <int LS>
__device__ __forceinline__ void group_d4(const GroupDesc &g, const uint32_t *__restrict__ zs,
                                         const double *__restrict__ cs, uint32_t Y, double (&dre)[4],
                                         double (&dim)[4])
{
#pragma unroll
    for (int i = 0; i < 4; i++) {
        dre[i] = 0.0;
        dim[i] = 0.0;
    }
    if constexpr (LS == kPatBit) {
        group_d4_part_pat(g.k0, g.kre, g.pat & 15, zs, cs, Y, dre);
        group_d4_part_pat(g.kre, g.k1, (g.pat >> 4) & 15, zs, cs, Y, dim);
    } else {
        group_d4_part<LS>(g.k0, g.kre, zs, cs, Y, dre);
        group_d4_part<LS>(g.kre, g.k1, zs, cs, Y, dim);
    }
}

// Sigma over tiles of 2^kSigL outputs: groups whose flip masks agree above
// bit kSigL form a class (ClassDesc, groups in class order), and for output
// tile t every group of class c reads its partner amplitudes psi[y ^ x] from
// the one tile t ^ xh_c.  That tile is staged in LDS once per class
// (double-buffered: the next class's tile is in flight in registers while
// this class is evaluated), so the state crosses HBM once per class instead
// of being gathered once per group.  A thread of the kSigNT-thread workgroup
// owns outputs tb | tid | 512 i (i < 4); D_g is evaluated at the partner
// index.  The workgroup takes tiles t0, t0 + dt, ... below ntiles, writes
// lam over them and returns the thread's share of <psi|lam> on them.  sp:
// two LDS buffers of 2^kSigL amplitudes; each tile ends with a workgroup
// barrier, after which sp may be reused.
constexpr int kSigL = 11;
constexpr int kSigNT = 512;

__device__ __forceinline__ double sigma_tiles(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                              uint32_t t0, uint32_t dt, uint32_t ntiles,
                                              const ClassDesc *__restrict__ classes, int ncls,
                                              const GroupDesc *__restrict__ groups, int G,
                                              const uint32_t *__restrict__ zs, const double *__restrict__ cs,
                                              double2 (*__restrict__ sp)[1u << kSigL])
{
    constexpr uint32_t T = 1u << kSigL;
    constexpr int IT = (int)(T / kSigNT);
    static_assert(IT == 4 && kSigNT == kItemStride, "four outputs 512 apart per thread");
    const uint32_t tid = threadIdx.x;
    const int lane = (int)(tid & 63u);
    double acc = 0.0;
    for (uint32_t t = t0; t < ntiles; t += dt) {
        const uint32_t tb = t << kSigL;
        double2 l[IT];
#pragma unroll
        for (int i = 0; i < IT; i++)
            l[i] = make_double2(0.0, 0.0);
        // the next partner tile, in flight in registers (four named values: an
        // array carried around the class loop was put in scratch memory)
        const uint32_t pb0 = (t ^ classes[0].xh) << kSigL;
        double2 p0 = psi[pb0 | tid], p1 = psi[pb0 | (tid + kSigNT)], p2 = psi[pb0 | (tid + 2 * kSigNT)],
                p3 = psi[pb0 | (tid + 3 * kSigNT)];
        // Group descriptors reach the wave 64 at a time, one per lane (coalesced
        // vector loads), and are broadcast by readlane: a scalar load per group
        // from a table larger than the scalar cache left the pass latency-bound
        // (~2500 clocks per group).  Strings are scalar loads (a readlane
        // broadcast of them costs three VALU per string, which measured slower).
        int gc = 0;
        uint32_t gxv = 0;
        int gk0v = 0, gkrev = 0, gk1v = 0, gpatv = 0;
        auto load_groups = [&](int g) __attribute__((always_inline)) {
            gc = g;
            const GroupDesc d = groups[min(g + lane, G - 1)];
            gxv = d.x;
            gk0v = d.k0;
            gkrev = d.kre;
            gk1v = d.k1;
            gpatv = d.pat;
        };
        load_groups(0);
        for (int c = 0; c < ncls; c++) {
            double2 *buf = sp[c & 1];
            buf[tid] = p0;
            buf[tid + kSigNT] = p1;
            buf[tid + 2 * kSigNT] = p2;
            buf[tid + 3 * kSigNT] = p3;
            const ClassDesc cd = classes[c];
            {
                // unconditional: the last class fetches its own tile again
                const uint32_t pb = (t ^ classes[c + 1 < ncls ? c + 1 : c].xh) << kSigL;
                p0 = psi[pb | tid];
                p1 = psi[pb | (tid + kSigNT)];
                p2 = psi[pb | (tid + 2 * kSigNT)];
                p3 = psi[pb | (tid + 3 * kSigNT)];
            }
            // buf is complete; its previous readers (class c - 2) passed the
            // barrier of class c - 1 before anyone writes it again
            __syncthreads();
            for (int g = cd.g0; g < cd.g1; g++) {
                if (g - gc >= 64)
                    load_groups(g);
                const int jg = g - gc;
                const uint32_t gx = (uint32_t)__builtin_amdgcn_readlane((int)gxv, jg);
                const int k0 = __builtin_amdgcn_readlane(gk0v, jg);
                const int kre = __builtin_amdgcn_readlane(gkrev, jg);
                const int k1 = __builtin_amdgcn_readlane(gk1v, jg);
                const int pat = __builtin_amdgcn_readlane(gpatv, jg);
                const uint32_t xl = gx & (T - 1u);
                const uint32_t Y = (tb | tid) ^ gx;
                double dre[IT], dimg[IT];
#pragma unroll
                for (int i = 0; i < IT; i++) {
                    dre[i] = 0.0;
                    dimg[i] = 0.0;
                }
                static_assert(kSigL - 2 == kPatBit, "items 2^(kSigL - 2) apart");
                group_d4_part_pat(k0, kre, pat & 15, zs, cs, Y, dre);
                if (k1 > kre) {
                    group_d4_part_pat(kre, k1, (pat >> 4) & 15, zs, cs, Y, dimg);
#pragma unroll
                    for (int i = 0; i < IT; i++) {
                        const double2 b = buf[(tid + (uint32_t)i * kSigNT) ^ xl];
                        l[i].x += dre[i] * b.x - dimg[i] * b.y;
                        l[i].y += dre[i] * b.y + dimg[i] * b.x;
                    }
                } else {  // real phases only (every string of a real Hamiltonian)
#pragma unroll
                    for (int i = 0; i < IT; i++) {
                        const double2 b = buf[(tid + (uint32_t)i * kSigNT) ^ xl];
                        l[i].x += dre[i] * b.x;
                        l[i].y += dre[i] * b.y;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < IT; i++) {
            const uint32_t y = tb | (tid + (uint32_t)i * kSigNT);
            lam[y] = l[i];
            const double2 p = psi[y];
            acc += p.x * l[i].x + p.y * l[i].y;
        }
        __syncthreads();  // the last class's buffer is read before sp is written again
    }
    return acc;
}

} // namespace qf
