// Host-side helpers shared by the plan path (qf_device.hip) and the batched
// path (qf_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <string>
#include <vector>

#include "qf_common.h"
#include "qf_kernels.h"

#define QF_HIP(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            qf::raise(QF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

namespace qf {

// Fault injection for tests of the error paths: with the environment variable
// QF_INJECT_ALLOC_FAIL=1 every device allocation of the library fails with
// QF_E_NOMEM (read at each allocation, so a test can switch it on and off).
inline bool alloc_failure_injected()
{
    const char *v = std::getenv("QF_INJECT_ALLOC_FAIL");
    return v && v[0] == '1';
}

template <class T> T *dev_alloc(size_t count)
{
    void *p = nullptr;
    if (alloc_failure_injected())
        raise(QF_E_NOMEM, "hipMalloc: failure injected by QF_INJECT_ALLOC_FAIL");
    if (count == 0)
        count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        raise(QF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return (T *)p;
}

inline uint32_t hibit(uint32_t x) { return x ? 31u - (uint32_t)__builtin_clz(x) : 0u; }

// Reject masks with a bit at or above n.
void check_terms(const char *who, int n, const qf_term *t, int64_t K);

// Split a term list into fused runs (see qf_device.hip); tab_entries receives
// the total size of the runs' (cos, sin) tables.
std::vector<RunDesc> make_runs(const qf_term *T, int64_t K, int &tab_entries);

// Per-group descriptors and the reordered (z, signed c) arrays of a grouped
// Hamiltonian.
void build_groups(int n, const qf_term *H, const int64_t *goff, int64_t G, std::vector<GroupDesc> &gd,
                  std::vector<uint32_t> &zs, std::vector<double> &cs);

// Tables of the streamed sigma for workgroups of nt (256 or 512) threads:
// sub-classes, group words and lo-terms (see qf_device.hip).
void sigma_stream_tables(const std::vector<GroupDesc> &gd, const std::vector<uint32_t> &zs,
                         const std::vector<double> &cs, int nt, std::vector<SsCls> &cls,
                         std::vector<uint32_t> &words, std::vector<SsLo> &los);

// Greedy split of a run sequence into segments whose flip masks fit one set
// of B qubits containing qubits 0..q0-1 (see qf_device.hip), at most
// max_runs runs (0: no limit) and max_tab table entries each; appends the
// segments' LocalRuns to lr (cleared first).  A Segment with Q == 0 holds
// one run too wide for a sub-cube; its r0 indexes `runs`.
void build_segments(const std::vector<RunDesc> &runs, int n, int B, int q0, std::vector<Segment> &segs,
                    std::vector<LocalRun> &lr, int max_runs = 0, int max_tab = kSegTab);

// Two-run passes of a blocked reverse sweep over (segs, lr): one AdjPair per
// LocalRun, set on the first run undone of each pair (see qf_kernels.h).
std::vector<AdjPair> adjoint_pairs(const std::vector<Segment> &segs, const std::vector<LocalRun> &lr);

// Three-run passes of a blocked apply on 2^12 sub-cubes: one ApplyTriple per
// LocalRun (the caller copies the w0 flags into the flip runs' itm[1]).
std::vector<ApplyTriple> apply_triples(const std::vector<Segment> &segs, const std::vector<LocalRun> &lr);

} // namespace qf
