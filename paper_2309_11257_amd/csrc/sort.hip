// Stable least-significant-digit radix sort of 32-bit keys with a 32-bit
// payload (8-bit digits), column offsets, and small bookkeeping kernels.
//
// Each pass: (1) per-tile digit histograms, (2) an exclusive scan over the
// digit-major histogram table, (3) a stable scatter where a tile ranks its keys
// among the wave's lanes with the same digit (runs of lanes when the digits
// do not decrease, else a 64-lane match on the 8 digit bits) and per-wave
// counts in LDS.  Tiles are 4096 keys (256 threads x 16 rounds, round-major so that
// consecutive keys of a round sit in consecutive lanes).  The element count
// is read from device memory, so no host synchronisation is needed; the
// grid is sized for an upper bound.
#include "rt_internal.h"

#define RS_THREADS 256
#define RS_ITEMS 16
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define SCAN_CHUNK 4096

static int64_t rs_blocks(int64_t bound) { return bound > 0 ? (bound + RS_TILE - 1) / RS_TILE : 1; }

int64_t radix_hist_len(int64_t bound)
{
    const int64_t nb = rs_blocks(bound);
    const int64_t table = 256 * nb;
    const int64_t parts = (table + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return table + parts + 1;
}

// Lanes of the wave holding the same 8-bit digit as this lane (valid lanes
// are a prefix of the wave).  The keys arrive nearly sorted, so a wave's
// digits usually do not decrease from lane to lane; then equal digits are
// runs of neighbouring lanes and one shuffle and one ballot find them.
// Otherwise the digit is matched bit by bit with eight ballots.
__device__ inline unsigned long long digit_peers(uint32_t d, bool valid, int lane)
{
    const uint32_t prev = (uint32_t)__shfl_up((int)d, 1, 64);  // lane 0: its own
    if (__ballot(valid && lane > 0 && d < prev) == 0ull) {
        const unsigned long long vm = __ballot(valid);
        const unsigned long long heads = __ballot(valid && (lane == 0 || d != prev));
        const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0 .. lane (all 64 for lane 63)
        const int h = 63 - __clzll(heads & upto);             // this lane's run head (-1: invalid lane)
        const unsigned long long above = heads & ~upto;
        const int e = above ? __ffsll(above) - 1 : __popcll(vm);  // first lane after the run
        const unsigned long long lo = h > 0 ? (1ull << h) - 1ull : 0ull;
        const unsigned long long hi = e == 64 ? ~0ull : (1ull << e) - 1ull;
        return valid ? (hi & ~lo) : 0ull;
    }
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
        const bool b = (d >> bit) & 1u;
        const unsigned long long m = __ballot(b);
        peers &= b ? m : ~m;
    }
    return valid ? peers : 0ull;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t *__restrict__ keys, const int64_t *n_dev, int shift,
                                                        int64_t nblocks, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const int lane = tid & 63;
    // lanes holding the same digit are counted by their lowest lane (keys
    // arrive nearly sorted, so a wave usually holds one or two digits)
    uint32_t kt[RS_ITEMS];  // all of the tile's keys in flight at once
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t i = base + (int64_t)it * RS_THREADS + tid;
        kt[it] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t i = base + (int64_t)it * RS_THREADS + tid;
        const bool valid = i < n;
        const uint32_t d = valid ? (kt[it] >> shift) & 255u : 0u;
        const unsigned long long peers = digit_peers(d, valid, lane);
        if (valid && lane == __ffsll((long long)peers) - 1) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// block-wide exclusive scan helper (256 threads), returns the block total
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t t = tid >= off ? sh[tid - off] : 0u;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    total = sh[255];
    const uint32_t incl = sh[tid];
    __syncthreads();
    return incl - v;
}

// pass 1 of the scan: sum of each SCAN_CHUNK-long part of the table
__global__ void k_scan_reduce(const uint32_t *__restrict__ t, int64_t len, uint32_t *__restrict__ parts)
{
    __shared__ uint32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    uint32_t s = 0;
    for (int q = threadIdx.x; q < SCAN_CHUNK; q += 256) {
        const int64_t i = base + q;
        if (i < len) s += t[i];
    }
    uint32_t tot;
    block_excl_scan(s, sh, tot);
    if (threadIdx.x == 0) parts[blockIdx.x] = tot;
}

// pass 2: exclusive scan of the part sums (one block)
__global__ void k_scan_parts(uint32_t *parts, int64_t nparts)
{
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (int64_t b = 0; b < nparts; b += 256) {
        const int64_t i = b + threadIdx.x;
        const uint32_t v = i < nparts ? parts[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, sh, tot);
        if (i < nparts) parts[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

// pass 3: exclusive scan inside each part, offset by the part prefix
__global__ void k_scan_apply(uint32_t *__restrict__ t, int64_t len, const uint32_t *__restrict__ parts)
{
    __shared__ uint32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    const int per = SCAN_CHUNK / 256;  // 16 consecutive entries per thread
    uint32_t loc[SCAN_CHUNK / 256];
    uint32_t s = 0;
    for (int q = 0; q < per; q++) {
        const int64_t i = base + (int64_t)threadIdx.x * per + q;
        loc[q] = i < len ? t[i] : 0u;
        s += loc[q];
    }
    uint32_t tot;
    uint32_t run = parts[blockIdx.x] + block_excl_scan(s, sh, tot);
    for (int q = 0; q < per; q++) {
        const int64_t i = base + (int64_t)threadIdx.x * per + q;
        if (i < len) t[i] = run;
        run += loc[q];
    }
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                           uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           const int64_t *n_dev, int shift, int64_t nblocks,
                                                           const uint32_t *__restrict__ offs)
{
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    base_off[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    run[tid] = 0;
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // the tile's keys and values are loaded before the rounds, so that the
    // rounds (and their barriers) do not wait on global memory one by one
    uint32_t kt[RS_ITEMS], vt[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t i = base + (int64_t)it * RS_THREADS + tid;
        kt[it] = i < n ? kin[i] : 0u;
        vt[it] = i < n ? (vin ? vin[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t i = base + (int64_t)it * RS_THREADS + tid;
        const bool valid = i < n;
        const uint32_t key = kt[it];
        const uint32_t val = vt[it];
        const uint32_t d = (key >> shift) & 255u;
        const unsigned long long peers = digit_peers(d, valid, lane);
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        wcnt[0][tid] = 0;
        wcnt[1][tid] = 0;
        wcnt[2][tid] = 0;
        wcnt[3][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wave][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pos = base_off[d] + run[d] + rank;
            for (int w = 0; w < wave; w++) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

int64_t scan_tmp_len(int64_t len) { return (len + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

void scan_u32(uint32_t *t, int64_t len, uint32_t *parts, hipStream_t s)
{
    if (len <= 0) return;
    const int64_t nparts = (len + SCAN_CHUNK - 1) / SCAN_CHUNK;
    k_scan_reduce<<<(unsigned)nparts, 256, 0, s>>>(t, len, parts);
    k_scan_parts<<<1, 256, 0, s>>>(parts, nparts);
    k_scan_apply<<<(unsigned)nparts, 256, 0, s>>>(t, len, parts);
}

void radix_sort(const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out, uint32_t *vals_out, uint32_t *tk,
                uint32_t *tv, uint32_t *hist, const int64_t *n_dev, int64_t bound, int nbits, hipStream_t s)
{
    const int64_t nb = rs_blocks(bound);
    const int64_t table = 256 * nb;
    const int64_t nparts = (table + SCAN_CHUNK - 1) / SCAN_CHUNK;
    uint32_t *parts = hist + table;
    int npass = (nbits + 7) / 8;
    if (npass < 1) npass = 1;
    const uint32_t *ck = keys, *cv = vals;
    for (int p = 0; p < npass; p++) {
        const bool to_out = ((npass - 1 - p) % 2) == 0;
        uint32_t *ok = to_out ? keys_out : tk;
        uint32_t *ov = to_out ? vals_out : tv;
        const int shift = 8 * p;
        k_rs_hist<<<(unsigned)nb, RS_THREADS, 0, s>>>(ck, n_dev, shift, nb, hist);
        k_scan_reduce<<<(unsigned)nparts, 256, 0, s>>>(hist, table, parts);
        k_scan_parts<<<1, 256, 0, s>>>(parts, nparts);
        k_scan_apply<<<(unsigned)nparts, 256, 0, s>>>(hist, table, parts);
        k_rs_scatter<<<(unsigned)nb, RS_THREADS, 0, s>>>(ck, cv, ok, ov, n_dev, shift, nb, hist);
        ck = ok;
        cv = ov;
    }
}

// sorted keys refined by the level back to column keys
__global__ void k_colkey(uint32_t *__restrict__ skeys, const DevCounters *__restrict__ dc, uint32_t nl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_sorted) return;
    skeys[i] = skeys[i] / nl;
}

void launch_colkey(uint32_t *skeys, const DevCounters *dc, uint32_t nl, int64_t bound, hipStream_t s)
{
    if (bound <= 0) return;
    k_colkey<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(skeys, dc, nl);
}

static __device__ inline int64_t lower_key(const uint32_t *__restrict__ skeys, int64_t n, uint32_t c)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skeys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// column c occupies sorted positions [colstart[c], colstart[c+1]); removed
// volumes (keys >= ncol) follow at [colstart[ncol], n_sorted).
//
// Wave table of the single-precision step (wcol non-null): column c with
// volumes at [s, e) gets waves c + s / 64 + j, j < ceil((e - s) / 64), each of
// up to 64 consecutive volumes of that column; the next column's first wave
// is c + 1 + e / 64, which is never below this column's last wave plus one,
// so the columns' waves do not overlap and the gaps between them are marked
// empty.  Waves from ncol + colstart[ncol] / 64 on are beyond every column.
__global__ void k_colstart(const uint32_t *__restrict__ skeys, DevCounters *dc, uint32_t *__restrict__ colstart,
                           uint32_t *__restrict__ wcol, int ncol)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncol) return;
    const int64_t n = dc->n_sorted;
    const int64_t s = lower_key(skeys, n, (uint32_t)c);
    colstart[c] = (uint32_t)s;
    if (c == ncol) dc->n_active = s;
    if (wcol && c < ncol) {
        const int64_t e = lower_key(skeys, n, (uint32_t)c + 1u);
        const int64_t w0 = c + s / 64, w1 = w0 + (e - s + 63) / 64, wn = c + 1 + e / 64;
        for (int64_t w = w0; w < w1; w++) wcol[w] = (uint32_t)c;
        for (int64_t w = w1; w < wn; w++) wcol[w] = 0xffffffffu;
    }
}

// upper bound of the waves of the single-precision step: sum over columns of
// ceil(n_c / 64) <= n / 64 + ncol
int64_t wave_table_len(int64_t cap, int ncol) { return cap / 64 + ncol + 1; }

void launch_colstart(const uint32_t *skeys, DevCounters *dc, uint32_t *colstart, uint32_t *wcol, int ncol,
                     hipStream_t s)
{
    k_colstart<<<(unsigned)((ncol + 1 + 255) / 256), 256, 0, s>>>(skeys, dc, colstart, wcol, ncol);
}

__global__ void k_set_sorted(DevCounters *dc, int64_t n) { dc->n_sorted = n; }
__global__ void k_sorted_from_active(DevCounters *dc)
{
    dc->n_sorted = dc->n_active;
    dc->steps += 1;
}

void launch_set_sorted(DevCounters *dc, int64_t n, hipStream_t s) { k_set_sorted<<<1, 1, 0, s>>>(dc, n); }
void launch_sorted_from_active(DevCounters *dc, hipStream_t s) { k_sorted_from_active<<<1, 1, 0, s>>>(dc); }

__global__ void k_copy_n(const uint32_t *src, uint32_t *dst, const DevCounters *dc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < dc->n_sorted) dst[i] = src[i];
}

void launch_copy_n(const uint32_t *src, uint32_t *dst, const DevCounters *dc, int64_t bound, hipStream_t s)
{
    if (bound > 0) k_copy_n<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(src, dst, dc);
}
