// Dynamic batching of the ARA iterations (getConvergedTiles, updateSubset):
// the stable compaction of the active list and the end-of-iteration
// bookkeeping, shared by the kernel that runs them alone and the fused
// launches of the ARA iteration.
#pragma once

#include "tlr_internal.h"

namespace tlr {
namespace {

// ------------------------------------------------------- dynamic batching
// Stable compaction of the active list act_in (slots whose flag is set
// leave) into act_out, then refill from the waiting list, keeping at most
// s_max tiles; counters from counts_in to counts_out ([0] active, [1]
// waiting cursor).  act_out may be act_in (in place: writes never overtake
// reads, pos <= index, and every read of a chunk precedes its first
// barrier).  Run by one whole workgroup of 256 threads, 256 entries at a
// time: a slot's position among those kept is the count of kept entries
// before it, from a ballot per wave and the four wave totals.  With width
// set, *qmax receives the largest width[slot] over the slots kept (the
// refilled ones have not run: width 0).  The loads form three rounds: the
// counters, the list, the per-slot flags and widths.
__device__ inline void compact_active(const int* act_in, int* act_out, const int* counts_in,
                                      int* counts_out, const int* flag, const int* waiting,
                                      int nwaiting, int s_max, const int* width, int* qmax,
                                      int* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = counts_in[0], cursor = counts_in[1];
  int kept = 0, qm = 0;
  for (int base = 0; base < n; base += 256) {
    const int i = base + tid;
    const int slot = (i < n) ? act_in[i] : -1;
    int keep = 0;
    if (slot >= 0) {
      keep = flag[slot] ? 0 : 1;
      if (width && keep) qm = max(qm, width[slot]);
    }
    const unsigned long long mask = __ballot(keep);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(mask);
    __syncthreads();
    int pos = kept + before;
    for (int w = 0; w < wv; ++w) pos += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    if (keep) act_out[pos] = slot;
    kept += total;
  }
  const int take = max(0, min(min(n - kept, s_max - kept), nwaiting - cursor));
  for (int j = tid; j < take; j += blockDim.x) act_out[kept + j] = waiting[cursor + j];
  if (qmax) {
    for (int off = 32; off > 0; off >>= 1) qm = max(qm, __shfl_xor(qm, off));
    if (lane == 0) wsum[4 + wv] = qm;
  }
  __syncthreads();
  if (qmax) *qmax = max(max(wsum[4], wsum[5]), max(wsum[6], wsum[7]));
  if (tid == 0) {
    counts_out[0] = kept + take;
    counts_out[1] = cursor + take;
  }
  __syncthreads();
}

// End of an ARA iteration: compact and refill the active list into the next
// iteration's copy, then record the status word and the largest basis
// width among the slots on it (the host's bound for the next products).
// Every thread of a 256-thread workgroup calls it.
__device__ inline void ara_compact_body(const AraDev& D, const int* waiting, int nwaiting,
                                        int s_max, const int* info, int* host_out, int* host_res,
                                        int res_ints) {
  __shared__ int wsum[8];
  const int tid = threadIdx.x;
  const int n = D.counts[0];   // active at entry: the iteration that ran
  const int st = info ? *info : 0;
  int qm = 0;
  compact_active(D.act, D.act_next, D.counts, D.counts_next, D.flag, waiting, nwaiting, s_max,
                 D.qout, &qm, wsum);
  const int na = D.counts_next[0];
  if (tid == 0) {
    D.counts_next[3] = qm;
    D.counts_next[2] = st;
  }
  // the four counters also go straight to the host's read-back slot
  // (pinned memory, stores at system scope)
  if (host_out && tid < 4) {
    const int v = tid == 0 ? na : tid == 1 ? D.counts_next[1] : tid == 2 ? st : qm;
    __hip_atomic_store(host_out + tid, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  // the compaction that empties the list (n > 0 tiles ran, none is left)
  // publishes the per-slot results (basis widths and counters, res_ints
  // contiguous ints from D.q), so the host need not wait for the iteration
  // queued behind it; that spare iteration starts empty and writes nothing
  if (host_res && n > 0 && na == 0) {
    for (int e = tid; e < res_ints; e += 256)
      __hip_atomic_store(host_res + e, D.q[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace
}  // namespace tlr
