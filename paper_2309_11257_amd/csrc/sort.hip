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
#define RS_TILE_SHIFT 12
#define RS_TILE (RS_THREADS * RS_ITEMS)
static_assert(RS_TILE == (1 << RS_TILE_SHIFT), "tile size");
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

// ---------------------------------------------------------------------------
// Regrouping after a step.  The step writes each volume's new key at the
// volume's position in the previous regrouping, so the keys arrive in that
// order, and the stable sort by the new key is known in advance for all but
// the few volumes whose key changed: in each column the stayers (new key =
// previous column) keep their previous order, preceded by the volumes that
// moved in from earlier positions and followed by those that moved in from
// later ones (each group by position); removed volumes follow all columns,
// by reason and then position.  Stayers and removed volumes are placed by
// counting (tile prefix sums of the volumes that changed key), the volumes
// that changed column by a sort of each column's few arrivals.  The result
// is the permutation the radix sort produces.

// Per-tile counting in thread order: a tile's RS_ITEMS rounds of RS_THREADS
// positions (round-major, position base + round * RS_THREADS + thread); each
// wave's ballot count of a flag per round goes to LDS cnt[round][wave], after
// which a lane's exclusive prefix over the tile in position order is
// tile_prefix(): earlier rounds whole, then earlier waves of its round, then
// its lower lanes.
__device__ inline uint32_t tile_prefix(const uint32_t (*cnt)[4], int it, unsigned long long ball)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t pre = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    for (int r = 0; r < it; r++) pre += cnt[r][0] + cnt[r][1] + cnt[r][2] + cnt[r][3];
    for (int w = 0; w < wave; w++) pre += cnt[it][w];
    return pre;
}

// counts: volumes leaving each column, arriving in each column (and those
// arriving from earlier positions), changed keys per tile, removed volumes
// per tile and reason, and the tile prefix of changed keys at each column's
// first position
__global__ __launch_bounds__(RS_THREADS) void k_rg_classify(const uint32_t *__restrict__ key,
                                                            const uint32_t *__restrict__ sk_old,
                                                            const uint32_t *__restrict__ cs_old,
                                                            const int64_t *n_dev, uint32_t ncol, int64_t nb,
                                                            RegroupBufs rb)
{
    __shared__ uint32_t cnt[RS_ITEMS][4];
    __shared__ uint32_t rc[RK_NREASON];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < RK_NREASON) rc[tid] = 0u;
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    // every round's keys in flight at once: new key, previous key, and the
    // previous key of the position before (a column's first position)
    uint32_t kt[RS_ITEMS], ot[RS_ITEMS], pt[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        kt[it] = p < n ? key[p] : 0u;
        ot[it] = p < n ? sk_old[p] : 0u;
        pt[it] = (p < n && p > 0) ? sk_old[p - 1] : 0xffffffffu;
    }
    unsigned long long bl[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        bl[it] = __ballot(p < n && kt[it] != ot[it]);
        if (lane == 0) cnt[it][wave] = (uint32_t)__popcll(bl[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        if (p >= n) continue;
        const uint32_t k = kt[it], o = ot[it];
        if (o != pt[it]) rb.lpc[o] = tile_prefix(cnt, it, bl[it]);
        if (k != o) {
            atomicAdd(&rb.outc[o], 1u);
            if (k < ncol) {
                atomicAdd(&rb.inc[k], 1u);
                if ((uint32_t)p < cs_old[k]) atomicAdd(&rb.inlow[k], 1u);
            } else {
                atomicAdd(&rc[k - ncol], 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int r = 0; r < RS_ITEMS; r++) t += cnt[r][0] + cnt[r][1] + cnt[r][2] + cnt[r][3];
        rb.tmv[blockIdx.x] = t;
    }
    if (tid < RK_NREASON) rb.rtc[(int64_t)tid * nb + blockIdx.x] = rc[tid];
}

// Exclusive scans of three sequences in one pair of launches, in chunks of
// RG_CHUNK values: the columns' (new count, arrivals) packed in one word
// (both sums stay below 2^32) -> (column offset, arrival bucket offset); the
// changed keys per tile; the removed volumes per tile, reason-major.  The
// first launch sums each chunk, the second adds the sums of the chunks
// before it (a few dozen) and scans its own.
#define RG_CHUNK 4096
struct RgScan {
    const uint32_t *cs_old;
    uint32_t ncol;
    int64_t nb;
    RegroupBufs rb;
    int64_t b1, b2;  // first chunk of the tile and removed sequences
    __device__ int64_t seg_len(int sg) const { return sg == 0 ? ncol : (sg == 1 ? nb : RK_NREASON * nb); }
    __device__ uint64_t get(int sg, int64_t i) const
    {
        if (sg == 0) {
            const uint32_t stay = (cs_old[i + 1] - cs_old[i]) - rb.outc[i];
            return ((uint64_t)(stay + rb.inc[i]) << 32) | (uint64_t)rb.inc[i];
        }
        return sg == 1 ? rb.tmv[i] : rb.rtc[i];
    }
    __device__ void put(int sg, int64_t i, uint64_t v) const
    {
        if (sg == 0) {
            rb.cnew[i] = (uint32_t)(v >> 32);
            rb.mstart[i] = (uint32_t)v;
        } else if (sg == 1) {
            rb.tmv[i] = (uint32_t)v;
        } else {
            rb.rtc[i] = (uint32_t)v;
        }
    }
    __device__ void locate(int64_t b, int &sg, int64_t &c0, int64_t &first) const
    {
        sg = b < b1 ? 0 : (b < b2 ? 1 : 2);
        first = sg == 0 ? 0 : (sg == 1 ? b1 : b2);
        c0 = (b - first) * RG_CHUNK;
    }
};

__global__ __launch_bounds__(256) void k_rg_sreduce(RgScan sc, uint64_t *btot)
{
    __shared__ uint64_t sh[256];
    int sg;
    int64_t c0, first;
    sc.locate(blockIdx.x, sg, c0, first);
    const int64_t len = sc.seg_len(sg);
    uint64_t s = 0;
    for (int q = threadIdx.x; q < RG_CHUNK; q += 256)
        if (c0 + q < len) s += sc.get(sg, c0 + q);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) btot[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_rg_sapply(RgScan sc, const uint64_t *__restrict__ btot, DevCounters *dc)
{
    __shared__ uint64_t sh[256];
    int sg;
    int64_t c0, first;
    sc.locate(blockIdx.x, sg, c0, first);
    const int64_t len = sc.seg_len(sg);
    const int tid = threadIdx.x;
    uint64_t pre = 0;
    for (int64_t b = first; b < (int64_t)blockIdx.x; b++) pre += btot[b];
    // 16 consecutive values a thread
    constexpr int PER = RG_CHUNK / 256;
    uint64_t v[PER];
    uint64_t s = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = c0 + (int64_t)tid * PER + q;
        v[q] = i < len ? sc.get(sg, i) : 0ull;
        s += v[q];
    }
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t t = tid >= off ? sh[tid - off] : 0ull;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    uint64_t run = pre + sh[tid] - s;
    const uint64_t chunk_total = sh[255];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int64_t i = c0 + (int64_t)tid * PER + q;
        if (i < len) sc.put(sg, i, run);
        run += v[q];
    }
    // the last column chunk ends the column sequence: the active count
    if (sg == 0 && tid == 0 && c0 + RG_CHUNK >= len) {
        const uint32_t tot = (uint32_t)((pre + chunk_total) >> 32);
        sc.rb.cnew[sc.ncol] = tot;
        dc->n_active = (int64_t)tot;
    }
}

// per column: where its first stayer goes, less that stayer's count of
// changed keys before it (so that a stayer at p goes to base + p - (changed
// keys before p)); the leaving counts are cleared for the next regrouping
__global__ void k_rg_base(const uint32_t *__restrict__ cs_old, uint32_t ncol, RegroupBufs rb, uint32_t *base)
{
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const uint32_t x = cs_old[c];
    uint32_t bs = 0;
    if (cs_old[c + 1] > x) bs = rb.cnew[c] + rb.inlow[c] - x + rb.tmv[x >> RS_TILE_SHIFT] + rb.lpc[c];
    base[c] = bs;
    rb.outc[c] = 0u;
}

// stayers and removed volumes to their places, arrivals into their column's
// bucket (in no particular order)
__global__ __launch_bounds__(RS_THREADS) void k_rg_place(const uint32_t *__restrict__ key,
                                                         const uint32_t *__restrict__ sk_old,
                                                         const uint32_t *__restrict__ cbase,
                                                         const int64_t *n_dev, uint32_t ncol, int64_t nb,
                                                         RegroupBufs rb, uint32_t *__restrict__ perm,
                                                         uint32_t *__restrict__ sk_new)
{
    __shared__ uint32_t cnt[RS_ITEMS][4];
    __shared__ uint32_t rcnt[RK_NREASON][RS_ITEMS][4];
    __shared__ int anyrem;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) anyrem = 0;
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint32_t tpre = rb.tmv[blockIdx.x];  // changed keys before this tile
    uint32_t kt[RS_ITEMS], ot[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        kt[it] = p < n ? key[p] : 0u;
        ot[it] = p < n ? sk_old[p] : 0u;
    }
    uint32_t bt[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) bt[it] = cbase[ot[it]];
    unsigned long long bl[RS_ITEMS];
    bool rem_here = false;
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        bl[it] = __ballot(p < n && kt[it] != ot[it]);
        if (lane == 0) cnt[it][wave] = (uint32_t)__popcll(bl[it]);
        rem_here = rem_here || (p < n && kt[it] >= ncol);
    }
    if (__ballot(rem_here) != 0ull && lane == 0) anyrem = 1;
    __syncthreads();
    const bool rem_tile = anyrem != 0;
    if (rem_tile) {
        // removed volumes per reason, round and wave
#pragma unroll
        for (int it = 0; it < RS_ITEMS; it++) {
            const int64_t p = base + (int64_t)it * RS_THREADS + tid;
            for (int r = 0; r < RK_NREASON; r++) {
                const unsigned long long bm = __ballot(p < n && kt[it] == ncol + (uint32_t)r);
                if (lane == 0) rcnt[r][it][wave] = (uint32_t)__popcll(bm);
            }
        }
        __syncthreads();
    }
    const uint32_t nact = rb.cnew[ncol];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; it++) {
        const int64_t p = base + (int64_t)it * RS_THREADS + tid;
        if (p >= n) continue;
        const uint32_t k = kt[it], o = ot[it];
        if (k == o) {
            const uint32_t q = bt[it] + (uint32_t)p - (tpre + tile_prefix(cnt, it, bl[it]));
            perm[q] = (uint32_t)p;
            sk_new[q] = o;
        } else if (k < ncol) {
            const uint32_t slot = atomicAdd(&rb.mfill[k], 1u);
            rb.mbuf[rb.mstart[k] + slot] = (uint32_t)p;
        } else {
            // removed: after the active volumes, by reason, then position
            // (the lanes here are this round's removed volumes of the wave)
            const uint32_t r = k - ncol;
            const unsigned long long below = (1ull << lane) - 1ull;
            uint32_t q = 0;
            for (int rr = 0; rr < RK_NREASON; rr++) {
                const unsigned long long bm = __ballot(r == (uint32_t)rr);
                if (r == (uint32_t)rr) q = (uint32_t)__popcll(bm & below);
            }
            q += nact + rb.rtc[(int64_t)r * nb + blockIdx.x];
            for (int rr = 0; rr < it; rr++) q += rcnt[r][rr][0] + rcnt[r][rr][1] + rcnt[r][rr][2] + rcnt[r][rr][3];
            for (int w = 0; w < wave; w++) q += rcnt[r][it][w];
            perm[q] = (uint32_t)p;
            sk_new[q] = k;
        }
    }
}

// each column's arrivals by position (low ones before its stayers, high ones
// after), its offset and its waves in the single-precision wave table; one
// wave per column, the counters cleared for the next regrouping
__global__ __launch_bounds__(256) void k_rg_arrivals(const uint32_t *__restrict__ cs_old, uint32_t ncol, RegroupBufs rb,
                                                     uint32_t *__restrict__ perm, uint32_t *__restrict__ sk_new,
                                                     uint32_t *__restrict__ colstart, uint32_t *__restrict__ wcol)
{
    const int lane = threadIdx.x & 63;
    const uint32_t c = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (c > ncol) return;
    if (c == ncol) {
        if (lane == 0) colstart[ncol] = rb.cnew[ncol];
        return;
    }
    const uint32_t m = rb.inc[c], low = rb.inlow[c], s = rb.cnew[c], e = rb.cnew[c + 1];
    const uint32_t stay = e - s - m;
    const uint32_t *bk = rb.mbuf + rb.mstart[c];
    if (m > 0 && m <= 64) {
        // bitonic sort of the arrivals' positions across the wave
        uint32_t v = (uint32_t)lane < m ? bk[lane] : 0xffffffffu;
        for (int kk = 2; kk <= 64; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const uint32_t w = (uint32_t)__shfl_xor((int)v, j, 64);
                const bool asc = (lane & kk) == 0, lower = (lane & j) == 0;
                v = (lower == asc) ? min(v, w) : max(v, w);
            }
        if ((uint32_t)lane < m) {
            const uint32_t t = (uint32_t)lane, q = t < low ? s + t : s + stay + t;
            perm[q] = v;
            sk_new[q] = c;
        }
    } else if (m > 64) {
        // rank by counting (a column rarely receives more than a wave's worth)
        for (uint32_t a = lane; a < m; a += 64) {
            const uint32_t v = bk[a];
            uint32_t t = 0;
            for (uint32_t b = 0; b < m; b++) t += bk[b] < v ? 1u : 0u;
            const uint32_t q = t < low ? s + t : s + stay + t;
            perm[q] = v;
            sk_new[q] = c;
        }
    }
    if (lane == 0) {
        colstart[c] = s;
        rb.inc[c] = 0u;
        rb.inlow[c] = 0u;
        rb.mfill[c] = 0u;
    }
    if (wcol) {
        const int64_t w0 = (int64_t)c + s / 64, w1 = w0 + (e - s + 63) / 64, wn = (int64_t)c + 1 + e / 64;
        for (int64_t w = w0 + lane; w < w1; w += 64) wcol[w] = c;
        for (int64_t w = w1 + lane; w < wn; w += 64) wcol[w] = 0xffffffffu;
    }
}

int64_t regroup_tiles(int64_t bound) { return rs_blocks(bound); }

// chunk sums of the three scans and the per-column stayer bases
int64_t regroup_scratch_words(int64_t cap, int ncol)
{
    const int64_t nb = rs_blocks(cap);
    const int64_t chunks = (ncol + RG_CHUNK - 1) / RG_CHUNK + (nb + RG_CHUNK - 1) / RG_CHUNK +
                           (RK_NREASON * nb + RG_CHUNK - 1) / RG_CHUNK;
    return 2 * chunks + ncol;
}

void regroup_after_step(const uint32_t *key, const uint32_t *sk_old, const uint32_t *cs_old, const int64_t *n_dev,
                        int64_t bound, int ncol, RegroupBufs rb, uint32_t *perm, uint32_t *sk_new, uint32_t *cs_new,
                        uint32_t *wcol, DevCounters *dc, hipStream_t s)
{
    const int64_t nb = rs_blocks(bound);
    const int64_t c1 = (ncol + RG_CHUNK - 1) / RG_CHUNK, c2 = (nb + RG_CHUNK - 1) / RG_CHUNK,
                  c3 = (RK_NREASON * nb + RG_CHUNK - 1) / RG_CHUNK;
    RgScan sc{cs_old, (uint32_t)ncol, nb, rb, c1, c1 + c2};
    uint64_t *btot = (uint64_t *)rb.scratch;
    uint32_t *cbase = (uint32_t *)(btot + c1 + c2 + c3);
    k_rg_classify<<<(unsigned)nb, RS_THREADS, 0, s>>>(key, sk_old, cs_old, n_dev, (uint32_t)ncol, nb, rb);
    k_rg_sreduce<<<(unsigned)(c1 + c2 + c3), 256, 0, s>>>(sc, btot);
    k_rg_sapply<<<(unsigned)(c1 + c2 + c3), 256, 0, s>>>(sc, btot, dc);
    k_rg_base<<<(unsigned)((ncol + 255) / 256), 256, 0, s>>>(cs_old, (uint32_t)ncol, rb, cbase);
    k_rg_place<<<(unsigned)nb, RS_THREADS, 0, s>>>(key, sk_old, cbase, n_dev, (uint32_t)ncol, nb, rb, perm, sk_new);
    k_rg_arrivals<<<(unsigned)((ncol + 1 + 3) / 4), 256, 0, s>>>(cs_old, (uint32_t)ncol, rb, perm, sk_new, cs_new,
                                                                wcol);
}

// Level refinement of a regrouping: each column's volumes, in position order
// after the regrouping, stably sorted by level index (the radix sort's order
// for the key column x (nz + 1) + level, whose ties keep position order);
// one wave per column, a counting sort over the column's levels in LDS.  The
// level of a volume is its stored level (single precision) or floor(z / dz)
// clamped to 0 .. nz (double precision), as in the level keys.
#define RG_LVL_WAVES 4
__device__ inline uint32_t rg_level(uint32_t slot, const int32_t *lev, const double *z, double dz, int nz)
{
    if (lev) return (uint32_t)min(max(lev[slot], 0), nz);
    const double q = floor(z[slot] / dz);
    return q > (double)nz ? (uint32_t)nz : (q >= 0.0 ? (uint32_t)q : 0u);  // NaN gives 0
}

// lanes of the wave holding the same level as this lane, valid lanes a prefix:
// runs of neighbours when the levels do not decrease (one shuffle, one
// ballot), else a match on the level's bits
__device__ inline unsigned long long level_peers(uint32_t d, bool valid, int lane, int nbits)
{
    const uint32_t prev = (uint32_t)__shfl_up((int)d, 1, 64);
    if (__ballot(valid && lane > 0 && d < prev) == 0ull) {
        const unsigned long long vm = __ballot(valid);
        const unsigned long long heads = __ballot(valid && (lane == 0 || d != prev));
        const unsigned long long upto = (2ull << lane) - 1ull;
        const int h = 63 - __clzll(heads & upto);
        const unsigned long long above = heads & ~upto;
        const int e = above ? __ffsll(above) - 1 : __popcll(vm);
        const unsigned long long lo = h > 0 ? (1ull << h) - 1ull : 0ull;
        const unsigned long long hi = e == 64 ? ~0ull : (1ull << e) - 1ull;
        return valid ? (hi & ~lo) : 0ull;
    }
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < nbits; bit++) {
        const bool b = (d >> bit) & 1u;
        const unsigned long long m = __ballot(b);
        peers &= b ? m : ~m;
    }
    return valid ? peers : 0ull;
}

__global__ __launch_bounds__(64 * RG_LVL_WAVES) void k_rg_levels(const uint32_t *__restrict__ pin,
                                                                 uint32_t *__restrict__ pout,
                                                                 const uint32_t *__restrict__ colstart, uint32_t ncol,
                                                                 const int32_t *__restrict__ lev,
                                                                 const double *__restrict__ z, double dz, int nz)
{
    extern __shared__ uint32_t lvl_bins[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nzp = nz + 1;
    uint32_t *bins = lvl_bins + wave * nzp;
    const uint32_t c = blockIdx.x * RG_LVL_WAVES + wave;
    if (c >= ncol) return;
    const uint32_t s = colstart[c], e = colstart[c + 1];
    if (e - s <= 1) {
        if (e > s && lane == 0) pout[s] = pin[s];
        return;
    }
    int nbits = 1;
    while ((1 << nbits) <= nz) nbits++;
    for (int q = lane; q < nzp; q += 64) bins[q] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // counts per level
    for (uint32_t j0 = s; j0 < e; j0 += 64) {
        const uint32_t j = j0 + lane;
        if (j < e) atomicAdd(&bins[rg_level(pin[j], lev, z, dz, nz)], 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // exclusive prefix over the levels, 64 at a time
    uint32_t carry = 0;
    for (int q0 = 0; q0 < nzp; q0 += 64) {
        const int q = q0 + lane;
        const uint32_t v = q < nzp ? bins[q] : 0u;
        uint32_t incl = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl += t;
        }
        if (q < nzp) bins[q] = carry + incl - v;
        carry += (uint32_t)__shfl((int)incl, 63, 64);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // place in position order: the rank among the chunk's lanes of the same
    // level, after the earlier chunks' (the bins advance by the run head)
    const unsigned long long below = (1ull << lane) - 1ull;
    for (uint32_t j0 = s; j0 < e; j0 += 64) {
        const uint32_t j = j0 + lane;
        const bool valid = j < e;
        const uint32_t slot = valid ? pin[j] : 0u;
        const uint32_t d = valid ? rg_level(slot, lev, z, dz, nz) : 0u;
        const unsigned long long peers = level_peers(d, valid, lane, nbits);
        const uint32_t base = valid ? bins[d] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            pout[s + base + (uint32_t)__popcll(peers & below)] = slot;
            if (lane == __ffsll((long long)peers) - 1) bins[d] = base + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

void regroup_levels(const uint32_t *pin, uint32_t *pout, const uint32_t *colstart, int ncol, const int32_t *lev,
                    const double *z, double dz, int nz, hipStream_t s)
{
    const size_t smem = sizeof(uint32_t) * (size_t)RG_LVL_WAVES * (size_t)(nz + 1);
    k_rg_levels<<<(unsigned)((ncol + RG_LVL_WAVES - 1) / RG_LVL_WAVES), 64 * RG_LVL_WAVES, smem, s>>>(
        pin, pout, colstart, (uint32_t)ncol, lev, z, dz, nz);
}

// the removed volumes' range [colstart[ncol], n) unchanged from pin to pout
__global__ void k_copy_removed(const uint32_t *__restrict__ pin, uint32_t *__restrict__ pout,
                               const uint32_t *__restrict__ cs_end, const int64_t *__restrict__ n_dev)
{
    const int64_t n = *n_dev;
    for (int64_t j = (int64_t)*cs_end + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        pout[j] = pin[j];
}

void copy_removed(const uint32_t *pin, uint32_t *pout, const uint32_t *cs_end, const int64_t *n_dev, hipStream_t s)
{
    k_copy_removed<<<256, 256, 0, s>>>(pin, pout, cs_end, n_dev);
}
