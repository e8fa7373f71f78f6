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
    int32_t q0;      // Q contains qubits 0 .. q0-1 (plans: kApplyQ0 / kAdjQ0; batched: 6; at most B)
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
constexpr int kAdjRuns = 20;       // runs of one blocked reverse-sweep segment (per-wave sums in LDS)
constexpr int kAdjTab = 256;       // (cos, sin) entries of one blocked reverse-sweep segment
constexpr int kPoolRuns = 28;      // runs of one read-only (pool) sweep segment: no tables staged
// Qubits 0 .. q0-1 are in every plan segment's set Q: rows of 2^q0
// amplitudes are contiguous in HBM.  Fewer fixed qubits leave more of Q for
// the runs' flip masks, so a segment holds more runs and the state makes
// fewer passes (24q UCCSD sweep, 2^11 sub-cubes: 217 segments at q0 = 6, 171
// at 3; 28q apply, 2^12: 122 at 6, 96 at 4); a row stays one or more whole
// 128-byte cache lines.  At most 8 qubits of Q lie above q0, so the row
// offsets of a sub-cube take 2^8 entries.
constexpr int kApplyQ0 = 4;
constexpr int kAdjQ0 = 3;
constexpr int kMaxHoff = 256;

struct LocalRun {
    uint32_t x, hbit, z0, a0;       // local flip mask, its highest bit, local z0, i^a0
    uint32_t b[kMaxRank];           // local GF(2) basis masks (zero beyond the rank)
    uint32_t z0f;                   // full-space z0
    uint32_t bf[kMaxRank];          // full-space basis masks
    int32_t r, tab;
    int32_t k0, m;                  // the run's strings (as in RunDesc)
    uint8_t e[kMaxRun];
    int8_t s[kMaxRun];
    uint32_t itm[2];                // per-item table-index and parity parts; a flip run
                                    // uses itm[0] only, and the blocked apply's runs
                                    // carry their ApplyTriple flags in itm[1]
};
static_assert(kMaxRun == 8, "e and s of a LocalRun fill one 64-bit word each");

// Reverse sweep, two runs per LDS pass: run A (LocalRun r) and run B (r - 1)
// of one segment, both flip runs of rank <= 3 with different flip masks and
// a0 odd.  Set on A's index (w0 bit 0); the kernel walks a segment's runs
// from the last and takes a pair wherever its run carries the flag.  Every
// uniform quantity of the pass is precomputed:
//   w0:   1 | plo << 8 | phi << 16, the two bits opened in the thread index
//         (the highest bit of xA and of xB reduced by xA);
//   bits: run A in bits 0..7, run B in bits 8..15: the table-index offset of
//         the second pair (3 bits: coordinates of xB for A, of xA for B), its
//         Z-parity offset (bit 3), par(x & z0) (bit 4), m >> 1 with m = a0 + 1
//         (bit 5) and the sign of q against the rotation's (bit 6);
//   tabs: the two runs' table offsets in the segment's table (A low half).
struct AdjPair {
    uint32_t w0, xA, xB;
    uint32_t bA[3], bB[3];
    uint32_t z0A, z0B;
    uint32_t bits, tabs;
    uint32_t pad[3];
};
static_assert(sizeof(AdjPair) == 64, "one scalar load of 16 dwords");

// Blocked apply, three runs per LDS pass (sub-cubes of 2^12 with 512
// threads: 8 amplitudes per thread, one coset of span(x0, x1, x2)).  Runs
// r, r + 1, r + 2 of a segment, flip runs of rank <= 3 with a0 odd and
// linearly independent flip masks.  The record sits on the first run
// (w0 bit 0, read by the forward walk); the last run carries w0 = 2 (read by
// the inverse walk, which then reads the record two runs back).  The same two
// flags are copied into the runs' LocalRun::itm[1], where the kernel tests
// them.
//   w0:   1 | s0 << 8 | s1 << 16 | s2 << 24, the three bits opened in the
//         thread index (the pivots of the echelon form of x0, x1, x2);
//   bits[j]: for run j and its two partner runs k1 < k2: the coordinates of
//         x_k1 (bits 0..2) and x_k2 (3..5), par(x_k1 & z0_j) (6),
//         par(x_k2 & z0_j) (7), par(x_j & z0_j) (8) and m >> 1 with
//         m = a0 + 3 (9);
//   tabs: the three runs' table offsets in the segment's table (10 bits each).
struct ApplyTriple {
    uint32_t w0;
    uint32_t x[3];
    uint32_t b[3][3];
    uint32_t z0[3];
    uint32_t bits[3];
    uint32_t tabs;
    uint32_t pad[12];
};
static_assert(sizeof(ApplyTriple) == 128, "scalar loads of whole records");

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

// Wavefront sums of 8 values per lane, all exchanges register moves (the
// gfx950 lane swaps and DPP), none through the LDS crossbar.  Two
// transposing steps with the two-operand lane swaps halve the values per
// lane with no selects: a permlane32 swap of values k and k + 4 leaves lanes
// 0..31 with value k summed over lane bit 5 and lanes 32..63 with value
// k + 4, then a permlane16 swap of k and k + 2 does the same over lane bit 4.
// A row rotation by 8 (keep one value, send the other) takes bit 3, and
// three in-row exchanges (quad_perm xor 1, xor 2, then the half-row mirror,
// which pairs the two quads of each half-row) add bits 0, 1 and 2.  Lane l
// then holds value sum8_index(l) = l >> 3 (its bits 5, 4, 3 = the value's
// bits 2, 1, 0); lanes with bits 0..2 clear (sum8_writer) hand the 8 totals
// on.  The order of additions is fixed.
__device__ __forceinline__ int sum8_index(int lane) { return lane >> 3; }

__device__ __forceinline__ bool sum8_writer(int lane) { return (lane & 7) == 0; }

// Every DPP control used here (quad_perm, row_ror, row_half_mirror, with
// all rows and banks enabled) reads a lane inside the same row, so no lane
// falls back to the old value and none needs to be supplied (bound_ctrl).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xb1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4e;        // quad_perm [2, 3, 0, 1]
constexpr int kDppRor8 = 0x128;       // row_ror:8
constexpr int kDppHalfMirror = 0x141; // row_half_mirror

// lanes 0..31: a(l) + a(l + 32); lanes 32..63: b(l - 32) + b(l).  The
// permlane32 swap trades the upper half of its first operand for the lower
// half of its second, so the two results are (a lo | b lo) and (a hi | b hi).
__device__ __forceinline__ double swap_add32(double a, double b)
{
    const auto pl = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double((int)ph[0], (int)pl[0]) + __hiloint2double((int)ph[1], (int)pl[1]);
}

// per pair of 16-lane rows (2j, 2j + 1): row 2j gets a(l) + a(l + 16), row
// 2j + 1 gets b(l - 16) + b(l) (the permlane16 swap trades the odd rows of
// its first operand for the even rows of its second)
__device__ __forceinline__ double swap_add16(double a, double b)
{
    const auto pl = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double((int)ph[0], (int)pl[0]) + __hiloint2double((int)ph[1], (int)pl[1]);
}

__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane)
{
    double w[4], x[2];
#pragma unroll
    for (int k = 0; k < 4; k++)
        w[k] = swap_add32(v[k], v[k + 4]);
#pragma unroll
    for (int k = 0; k < 2; k++)
        x[k] = swap_add16(w[k], w[k + 2]);
    const bool b3 = (lane >> 3) & 1;
    const double send = b3 ? x[0] : x[1];
    const double keep = b3 ? x[1] : x[0];
    double h = keep + dpp_f64<kDppRor8>(send);
    h += dpp_f64<kDppXor1>(h);
    h += dpp_f64<kDppXor2>(h);
    h += dpp_f64<kDppHalfMirror>(h);
    return h;
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

// ---------------------------------------------------------------- multi-run passes
// One run of an ApplyTriple on the thread's coset held in v (v[i] is
// c0 ^ (i & 1) x0 ^ (i >> 1 & 1) x1 ^ (i >> 2) x2): run J's pairs are
// (v[i], v[i | 2^J]) for the four i with bit J clear; each pair's table index
// and Z-parity differ from those of c0 by the tabulated offsets of its
// partner-run coordinates.  u0, p0: table index and rotation sign bit at c0.
template <int J>
__device__ __forceinline__ void triple_run(double2 (&v)[8], const double2 *tb, uint32_t u0, uint32_t p0,
                                           uint32_t bits)
{
    constexpr int K1 = J == 0 ? 1 : 0, K2 = J == 2 ? 1 : 2;
    const uint32_t d1 = bits & 7u, d2 = (bits >> 3) & 7u, px = ((bits >> 8) & 1u) << 31;
    double2 cs[4];
#pragma unroll
    for (int t = 0; t < 4; t++)
        cs[t] = tb[u0 ^ ((t & 1) ? d1 : 0u) ^ ((t & 2) ? d2 : 0u)];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int i = ((t & 1) << K1) | ((t >> 1) << K2);
        const uint32_t P1 = (p0 ^ ((t & 1) ? bits >> 6 : 0u) ^ ((t & 2) ? bits >> 7 : 0u)) << 31;
        rot_pair<false>(cs[t].x, flip31(cs[t].y, P1), flip31(cs[t].y, P1 ^ px), v[i], v[i | (1 << J)]);
    }
}

// Three consecutive runs applied in one LDS pass (ApplyTriple), in order
// (FWD) or as their inverses in reverse order; pbz: the three runs' entries
// of the sub-cube's fixed-bit parities.
template <bool FWD>
__device__ __forceinline__ void apply_three(double2 *st, const double2 *stab, const ApplyTriple &T,
                                            const uint32_t *pbz, uint32_t tid)
{
    const uint32_t c0 = insert0(insert0(insert0(tid, (T.w0 >> 8) & 31u), (T.w0 >> 16) & 31u), T.w0 >> 24);
    // (the addresses are formed again for the stores: 8 fewer live registers)
    auto yi = [&](int i) { return c0 ^ ((i & 1) ? T.x[0] : 0u) ^ ((i & 2) ? T.x[1] : 0u) ^ ((i & 4) ? T.x[2] : 0u); };
    double2 v[8];
#pragma unroll
    for (int i = 0; i < 8; i++)
        v[i] = st[yi(i)];
    uint32_t u0[3], p0[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const uint32_t pb = pbz[j];
        u0[j] = (pb & 63u) ^ par(c0 & T.b[j][0]) ^ (par(c0 & T.b[j][1]) << 1) ^ (par(c0 & T.b[j][2]) << 2);
        // the inverse negates the angle: one more sign on every pair
        p0[j] = par(c0 & T.z0[j]) ^ (pb >> 6) ^ (T.bits[j] >> 9) ^ (FWD ? 0u : 1u);
    }
    const double2 *tb0 = stab + (T.tabs & 1023u), *tb1 = stab + ((T.tabs >> 10) & 1023u),
                  *tb2 = stab + (T.tabs >> 20);
    if (FWD) {
        triple_run<0>(v, tb0, u0[0], p0[0], T.bits[0]);
        triple_run<1>(v, tb1, u0[1], p0[1], T.bits[1]);
        triple_run<2>(v, tb2, u0[2], p0[2], T.bits[2]);
    } else {
        triple_run<2>(v, tb2, u0[2], p0[2], T.bits[2]);
        triple_run<1>(v, tb1, u0[1], p0[1], T.bits[1]);
        triple_run<0>(v, tb0, u0[0], p0[0], T.bits[0]);
    }
#pragma unroll
    for (int i = 0; i < 8; i++)
        st[yi(i)] = v[i];
}

// *p += v for an LDS word that only this lane adds to: the LDS add returns
// nothing, so the lane does not wait for the old value (the order of the
// additions is the lane's program order)
__device__ __forceinline__ void wave_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One flip-run pair of the reverse sweep on registers: q of the pair (a, b)
// (phi) and (la, lb) (lambda) as in adjoint_pairs, then the pair undone.
template <bool SW>
__device__ __forceinline__ double adjoint_one_pair(double2 &a, double2 &b, double2 &la, double2 &lb, double2 cs,
                                                   uint32_t P1, uint32_t px31, uint32_t dq31)
{
    const uint32_t P2 = P1 ^ px31;
    const double f1 = SW ? lb.x * a.y - lb.y * a.x : lb.x * a.x + lb.y * a.y;
    const double f2 = SW ? la.x * b.y - la.y * b.x : la.x * b.x + la.y * b.y;
    const double q = flip31(f1, P1 ^ dq31) + flip31(f2, P2 ^ dq31);
    const double s1 = flip31(cs.y, P1), s2 = flip31(cs.y, P2);
    rot_pair<SW>(cs.x, s1, s2, a, b);
    rot_pair<SW>(cs.x, s1, s2, la, lb);
    return q;
}

// Two consecutive runs undone in one LDS pass (an AdjPair).  The sub-cube
// splits into the 2^(B-2) cosets {c0, c0 ^ xA, c0 ^ xB, c0 ^ xA ^ xB} of
// span(xA, xB); thread t holds coset t (c0: zeros opened at the pair's two
// pivot bits) of phi and lambda in registers, so both runs' pairs are its own
// and no barrier separates them.  Run A's pairs are (c0, c0 ^ xA) and
// (c2, c2 ^ xA) with c2 = c0 ^ xB, run B's (c0, c2) and (c1, c1 ^ xB) with
// c1 = c0 ^ xA.  Table index and Z-parity are affine in y, so each second
// pair differs from the first by the tabulated uniform offsets.  Both runs'
// Walsh sums of the wave are added to (ADD) or stored in sumA and sumB
// (their 8 entries).
template <bool ADD>
__device__ __forceinline__ void adjoint_two(double2 *sp, double2 *sl, const double2 *stab, const AdjPair &pr,
                                            uint32_t pbzA, uint32_t pbzB, uint32_t tid, int lane, double *sumA,
                                            double *sumB)
{
    const uint32_t plo = (pr.w0 >> 8) & 31u, phi = (pr.w0 >> 16) & 31u;
    const uint32_t c0 = insert0(insert0(tid, plo), phi);
    const uint32_t c1 = c0 ^ pr.xA, c2 = c0 ^ pr.xB, c3 = c2 ^ pr.xA;
    const uint32_t bA = pr.bits & 0xffu, bB = (pr.bits >> 8) & 0xffu;
    const double2 *tbA = stab + (pr.tabs & 0xffffu), *tbB = stab + (pr.tabs >> 16);
    const uint32_t uA0 = (pbzA & 63u) ^ par(c0 & pr.bA[0]) ^ (par(c0 & pr.bA[1]) << 1) ^ (par(c0 & pr.bA[2]) << 2);
    const uint32_t uB0 = (pbzB & 63u) ^ par(c0 & pr.bB[0]) ^ (par(c0 & pr.bB[1]) << 1) ^ (par(c0 & pr.bB[2]) << 2);
    const uint32_t uA1 = uA0 ^ (bA & 7u), uB1 = uB0 ^ (bB & 7u);
    const double2 csA0 = tbA[uA0], csA1 = tbA[uA1], csB0 = tbB[uB0], csB1 = tbB[uB1];
    double2 a0 = sp[c0], a1 = sp[c1], a2 = sp[c2], a3 = sp[c3];
    double2 l0 = sl[c0], l1 = sl[c1], l2 = sl[c2], l3 = sl[c3];
    const uint32_t PA0 = (par(c0 & pr.z0A) ^ (pbzA >> 6) ^ (bA >> 5)) << 31;
    const uint32_t PA1 = PA0 ^ ((bA >> 3) << 31);
    const uint32_t PB0 = (par(c0 & pr.z0B) ^ (pbzB >> 6) ^ (bB >> 5)) << 31;
    const uint32_t PB1 = PB0 ^ ((bB >> 3) << 31);
    // Run A, then run B one pair at a time, each B pair stored as soon as it
    // is final; the Walsh sums and wave reductions follow with only the four
    // q values live.  (Scheduling fences between the steps: interleaved, the
    // steps hold more than the 128 registers of four waves per SIMD.)
    double qA[2], qB[2];
    {
        const uint32_t px = (bA >> 4) << 31, dq = (bA >> 6) << 31;
        qA[0] = adjoint_one_pair<false>(a0, a1, l0, l1, csA0, PA0, px, dq);
        __builtin_amdgcn_sched_barrier(0);
        qA[1] = adjoint_one_pair<false>(a2, a3, l2, l3, csA1, PA1, px, dq);
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        const uint32_t px = (bB >> 4) << 31, dq = (bB >> 6) << 31;
        qB[0] = adjoint_one_pair<false>(a0, a2, l0, l2, csB0, PB0, px, dq);
        sp[c0] = a0;
        sp[c2] = a2;
        sl[c0] = l0;
        sl[c2] = l2;
        __builtin_amdgcn_sched_barrier(0);
        qB[1] = adjoint_one_pair<false>(a1, a3, l1, l3, csB1, PB1, px, dq);
        sp[c1] = a1;
        sp[c3] = a3;
        sl[c1] = l1;
        sl[c3] = l3;
    }
    __builtin_amdgcn_sched_barrier(0);
    // (no branch before both sums: a branch lets the compiler sink run B's
    // q past it and keep all eight amplitudes live through the first sum)
    double w[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        double acc[kMaxRun];
#pragma unroll
        for (int k = 0; k < kMaxRun; k++)
            acc[k] = -0.0;
        const uint32_t du[2] = {0u, h ? uB0 ^ uB1 : uA0 ^ uA1};
        walsh_add<2>(acc, h ? uB0 : uA0, du, h ? qB : qA);
        w[h] = wave_sum8(acc, lane);
    }
    if (sum8_writer(lane)) {
        if (ADD) {
            wave_add(&sumA[sum8_index(lane)], w[0]);
            wave_add(&sumB[sum8_index(lane)], w[1]);
        } else {
            sumA[sum8_index(lane)] = w[0];
            sumB[sum8_index(lane)] = w[1];
        }
    }
}

// ---------------------------------------------------------------- sigma, streamed
// lambda = H psi with the signs evaluated at the output index.  For a string
// of real phase omega(y ^ x) = omega(y), for one of imaginary phase
// omega(y ^ x) = -omega(y), so lambda[y] = sum_g (dre_g(y) - i dim_g(y))
// psi[y ^ x_g] with dre, dim the sums of the folded coefficients times
// (-1)^popcount(y & z) (host tables carry the imaginary part negated).
// Output tiles of 2^11: with y = t 2^11 | tid | i NT (NT threads, NI = 2^11 /
// NT items) the sign splits into (-1)^popcount(t & z_hi), uniform over the
// tile, (-1)^popcount(tid & z_lo) per thread and (-1)^popcount(i & p),
// p = z_lo >> log2(NT), fixed per item.  So strings of a group part with
// equal z_lo merge per tile into one lo-term of coefficient
// C(t) = sum c (-1)^popcount(t & z_hi), and lo-terms sorted by z_lo come in
// runs of equal p: a run sums a = sum C (-1)^popcount(tid & z_lo) once and
// adds +-a to the items' coefficients (uniform signs).
//
// The caller's workgroup owns one output tile at a time (t0, t0 + dt, ...)
// and walks the sub-classes (groups with the same flip bits above the tile,
// at most NT groups and NT lo-terms each).  For each it stages the partner
// tile t ^ xh in LDS, with one lo-term per thread (C(t) computed from the
// tabled strings) and one group word per thread; the next sub-class's tile,
// lo-term and group word are in flight in registers meanwhile.  Waves pull a
// group's lo-terms (at most 64) into lanes with one LDS read and broadcast
// them by readlane.  LDS: tile (2^11 amplitudes), wlo (NT entries), wgw (NT
// words); each sub-class ends with the workgroup at a barrier, after which
// they may be reused.  Returns the thread's share of Re <psi|lambda>.
constexpr int kSsL = 11;
constexpr int kSsGrp = 64;               // lo-terms per group (larger groups are cut)
constexpr uint32_t kSsFlush = 1u << 11;  // last lo-term of a run of equal p
constexpr uint32_t kSsImag = 1u << 12;   // lo-term of the imaginary part
constexpr uint32_t kSsOne = 1u << 14;    // group word: one run (pattern in bits 11..13)

struct SsLo {
    uint32_t zf;       // z_lo | kSsFlush | kSsImag
    uint32_t zhi[3];   // z >> 11 of up to three strings, as tile-index masks
    double c[3];       // their coefficients (0 where unused)
    double pad;
};

struct SsCls {
    uint32_t xh;       // partner tile t ^ xh
    int32_t g0, l0;    // first group word / lo-term
    int32_t ng, nl;    // counts, 1..NT
    int32_t pad[3];
};

// the NI item signs (-1)^popcount(i & p) as sign-bit words
template <int NI>
__device__ __forceinline__ void ss_signs(uint32_t p, uint32_t (&sg)[NI])
{
    const uint32_t m1 = p << 31, m2 = (p >> 1) << 31, m4 = (p >> 2) << 31;
    const uint32_t all[8] = {0u, m1, m2, m1 ^ m2, m4, m1 ^ m4, m2 ^ m4, m1 ^ m2 ^ m4};
#pragma unroll
    for (int i = 0; i < NI; i++)
        sg[i] = all[i];
}

// a = sum over the group's lo-terms k0 <= k < k1 (lanes of lch) of
// C (-1)^popcount(tid & z_lo), two at a time into two sums
__device__ __forceinline__ double ss_sum(const uint4 &lch, int nlo, uint32_t tid)
{
    double a = 0.0, a2 = 0.0;
    int k = 0;
    for (; k + 1 < nlo; k += 2) {
        const uint32_t z0 = (uint32_t)__builtin_amdgcn_readlane((int)lch.x, k);
        const uint32_t z1 = (uint32_t)__builtin_amdgcn_readlane((int)lch.x, k + 1);
        const double C0 = __hiloint2double(__builtin_amdgcn_readlane((int)lch.w, k),
                                           __builtin_amdgcn_readlane((int)lch.z, k));
        const double C1 = __hiloint2double(__builtin_amdgcn_readlane((int)lch.w, k + 1),
                                           __builtin_amdgcn_readlane((int)lch.z, k + 1));
        a = fma(pm_one((uint32_t)__popc(tid & z0) << 31), C0, a);
        a2 = fma(pm_one((uint32_t)__popc(tid & z1) << 31), C1, a2);
    }
    if (k < nlo) {
        const uint32_t z0 = (uint32_t)__builtin_amdgcn_readlane((int)lch.x, k);
        const double C0 = __hiloint2double(__builtin_amdgcn_readlane((int)lch.w, k),
                                           __builtin_amdgcn_readlane((int)lch.z, k));
        a = fma(pm_one((uint32_t)__popc(tid & z0) << 31), C0, a);
    }
    return a + a2;
}

template <int NT, bool IMAG>
__device__ __forceinline__ double sigma_stream(const double2 *__restrict__ psi, double2 *__restrict__ lam,
                                               uint32_t t0, uint32_t dt, uint32_t ntiles,
                                               const SsCls *__restrict__ cls, int ncls,
                                               const uint32_t *__restrict__ gwords, const SsLo *__restrict__ los,
                                               double2 *__restrict__ tile, uint4 *__restrict__ wlo,
                                               uint32_t *__restrict__ wgw)
{
    constexpr uint32_t T = 1u << kSsL;
    constexpr int NI = (int)(T / NT);
    constexpr int IS = NT == 256 ? 8 : 9;  // item i is bit IS and up of the tile index
    static_assert((NT == 256 && NI == 8) || (NT == 512 && NI == 4), "2^11 outputs per tile");
    // item rows read per step: all of them, or two halves of four (eight items:
    // fewer live registers)
    constexpr int NH = NI == 8 ? 4 : NI;
    const uint32_t tid = threadIdx.x, tid16 = tid << 4;
    const int lane = (int)(tid & 63u);
    double acc = 0.0;
    for (uint32_t t = t0; t < ntiles; t += dt) {
        double2 l[NI];
#pragma unroll
        for (int i = 0; i < NI; i++)
            l[i] = make_double2(0.0, 0.0);
        // sub-class in flight: its tile, lo-term and group word (raw loads;
        // named values: an array carried around the loop went to scratch)
        double2 p0, p1, p2, p3, p4, p5, p6, p7;
        uint32_t zfn, zh0, zh1, zh2, gwn;
        double c0, c1, c2;
        SsCls cn = cls[0];
        auto fetch = [&]() __attribute__((always_inline)) {
            const double2 *src = psi + ((size_t)(t ^ cn.xh) << kSsL) + tid;
            p0 = src[0];
            p1 = src[1u << IS];
            p2 = src[2u << IS];
            p3 = src[3u << IS];
            if constexpr (NI == 8) {
                p4 = src[4u << IS];
                p5 = src[5u << IS];
                p6 = src[6u << IS];
                p7 = src[7u << IS];
            }
            const SsLo &r = los[cn.l0 + min((int)tid, cn.nl - 1)];
            zfn = r.zf;
            zh0 = r.zhi[0];
            zh1 = r.zhi[1];
            zh2 = r.zhi[2];
            c0 = r.c[0];
            c1 = r.c[1];
            c2 = r.c[2];
            gwn = gwords[cn.g0 + min((int)tid, cn.ng - 1)];
        };
        fetch();
        for (int c = 0; c < ncls; c++) {
            const int ng = cn.ng;
            __syncthreads();  // the previous sub-class's LDS reads are done
            tile[tid] = p0;
            tile[tid + (1u << IS)] = p1;
            tile[tid + (2u << IS)] = p2;
            tile[tid + (3u << IS)] = p3;
            if constexpr (NI == 8) {
                tile[tid + (4u << IS)] = p4;
                tile[tid + (5u << IS)] = p5;
                tile[tid + (6u << IS)] = p6;
                tile[tid + (7u << IS)] = p7;
            }
            {
                const double C = flip(c0, par(t & zh0)) + flip(c1, par(t & zh1)) + flip(c2, par(t & zh2));
                wlo[tid] = make_uint4(zfn, 0u, (uint32_t)__double2loint(C), (uint32_t)__double2hiint(C));
                wgw[tid] = gwn;
            }
            __syncthreads();
            cn = cls[c + 1 < ncls ? c + 1 : c];
            fetch();  // unconditional: the last sub-class fetches itself again
            int jw = 0;
            uint4 lch = make_uint4(0u, 0u, 0u, 0u);
            uint32_t gch = 0u;
            for (int g = 0; g < ng; g++) {
                if ((g & 63) == 0)
                    gch = wgw[g + lane];
                const uint32_t gw = (uint32_t)__builtin_amdgcn_readlane((int)gch, g & 63);
                const int nlo = (int)(gw >> 16);
                // the group's lo-terms, one per lane (lanes past them read
                // entries that are not used)
                lch = wlo[min(jw + lane, NT - 1)];
                jw += nlo;
                // a group whose lo-terms all cancel on this tile adds nothing
                // (number-conserving Hamiltonians: ~20 % of group-tile pairs)
                {
                    const double Cl = __hiloint2double((int)lch.w, (int)lch.z);
                    const uint64_t nz = __builtin_amdgcn_ballot_w64(Cl != 0.0);
                    const uint64_t lm = nlo >= 64 ? ~0ull : ((1ull << nlo) - 1ull);
                    if (!(nz & lm))
                        continue;
                }
                const uint32_t base = tid16 ^ ((gw & (T - 1u)) << 4);
                auto row = [&](int i) __attribute__((always_inline)) {
                    return *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(tile) +
                                                              (base ^ ((uint32_t)i << (IS + 4))));
                };
                double2 b[NH];
#pragma unroll
                for (int i = 0; i < NH; i++)
                    b[i] = row(i);
                // the items' coefficients: dr + i di
                double dr[NI], di[IMAG ? NI : 1];
                if (!IMAG && (gw & kSsOne)) {
                    // one run (one phase part, one item pattern): sign its sum
                    const double a = ss_sum(lch, nlo, tid);
                    uint32_t sg[NI];
                    ss_signs<NI>((gw >> 11) & 7u, sg);
#pragma unroll
                    for (int i = 0; i < NI; i++)
                        dr[i] = pm_one(sg[i]) * a;
                } else {
#pragma unroll
                    for (int i = 0; i < NI; i++) {
                        dr[i] = 0.0;
                        if (IMAG)
                            di[IMAG ? i : 0] = 0.0;
                    }
                    double a = 0.0;
                    for (int k = 0; k < nlo; k++) {
                        const uint32_t zf = (uint32_t)__builtin_amdgcn_readlane((int)lch.x, k);
                        const double C = __hiloint2double(__builtin_amdgcn_readlane((int)lch.w, k),
                                                          __builtin_amdgcn_readlane((int)lch.z, k));
                        a = fma(pm_one((uint32_t)__popc(tid & zf) << 31), C, a);
                        if (zf & kSsFlush) {
                            uint32_t sg[NI];
                            ss_signs<NI>((zf >> IS) & 7u, sg);
                            if (IMAG && (zf & kSsImag)) {
#pragma unroll
                                for (int i = 0; i < NI; i++)
                                    di[IMAG ? i : 0] = fma(pm_one(sg[i]), a, di[IMAG ? i : 0]);
                            } else {
#pragma unroll
                                for (int i = 0; i < NI; i++)
                                    dr[i] = fma(pm_one(sg[i]), a, dr[i]);
                            }
                            a = 0.0;
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < NI; h += NH) {
                    if (h > 0) {
#pragma unroll
                        for (int i = 0; i < NH; i++)
                            b[i] = row(h + i);
                    }
#pragma unroll
                    for (int i = 0; i < NH; i++) {
                        l[h + i].x = fma(dr[h + i], b[i].x, l[h + i].x);
                        l[h + i].y = fma(dr[h + i], b[i].y, l[h + i].y);
                        if (IMAG) {
                            l[h + i].x = fma(-di[IMAG ? h + i : 0], b[i].y, l[h + i].x);
                            l[h + i].y = fma(di[IMAG ? h + i : 0], b[i].x, l[h + i].y);
                        }
                    }
                }
            }
        }
        const size_t tb = (size_t)t << kSsL;
#pragma unroll
        for (int i = 0; i < NI; i++) {
            const size_t y = tb + tid + ((uint32_t)i << IS);
            const double2 p = psi[y];
            lam[y] = l[i];
            acc += p.x * l[i].x + p.y * l[i].y;
        }
    }
    // the workgroup's last LDS reads are done before the caller reuses it
    __syncthreads();
    return acc;
}

} // namespace qf
