// Tallies of the volumes a sort put after the active ones (sorted key
// ncol + reason): count per reason, their total wave action, and the
// smallest id among those deactivated as non-finite or degenerate.  The removed
// range is cut into TALLY_BLOCKS contiguous chunks, one per workgroup; each
// sums its chunk with a fixed tree and the chunk sums are added in chunk
// order, so the total does not depend on scheduling.  Counts are integers.
#pragma once
#include "rt_internal.h"

#define TALLY_BLOCKS 256

// WF::W(slot), WF::id(slot): wave action and id of the volume in storage slot `slot`
template <class WF>
__global__ __launch_bounds__(256) void k_tally_part(Grid g, WF wf, const uint32_t *__restrict__ perm,
                                                    const uint32_t *__restrict__ skeys, DevCounters *dc,
                                                    double *__restrict__ part)
{
    __shared__ double sw[256];
    __shared__ int cnt[RK_NREASON];
    __shared__ unsigned long long badk;
    const int tid = threadIdx.x;
    if (tid < RK_NREASON) cnt[tid] = 0;
    if (tid == 0) badk = 0ull;
    __syncthreads();
    const int64_t a = dc->n_active, e = dc->n_sorted;
    const int64_t chunk = (e - a + TALLY_BLOCKS - 1) / TALLY_BLOCKS;
    const int64_t b0 = a + (int64_t)blockIdx.x * chunk, b1 = min(e, b0 + chunk);
    double w = 0.0;
    for (int64_t i = b0 + tid; i < b1; i += 256) {
        const int reason = (int)(skeys[i] - (uint32_t)g.ncol);
        if (reason >= 0 && reason < RK_NREASON) atomicAdd(&cnt[reason], 1);
        if (reason != RK_INVALID && reason != RK_MERGED) w += wf.W(perm[i]);
        if (reason == RK_INVALID) atomicMax(&badk, ~(unsigned long long)wf.id(perm[i]));
    }
    sw[tid] = w;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) sw[tid] += sw[tid + off];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = sw[0];
    if (tid < RK_NREASON && cnt[tid]) atomicAdd((unsigned long long *)&dc->removed[tid], (unsigned long long)cnt[tid]);
    if (tid == 0 && badk) atomicMax((unsigned long long *)&dc->bad_key, badk);
}

static __global__ void k_tally_final(const double *__restrict__ part, DevCounters *dc)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < TALLY_BLOCKS; b++) s += part[b];
    dc->removed_W += s;
}

template <class WF>
inline void launch_tally_k(const Grid &g, const WF &wf, const uint32_t *perm, const uint32_t *skeys,
                           DevCounters *dc, double *part, hipStream_t s)
{
    k_tally_part<WF><<<TALLY_BLOCKS, 256, 0, s>>>(g, wf, perm, skeys, dc, part);
    k_tally_final<<<1, 64, 0, s>>>(part, dc);
}
