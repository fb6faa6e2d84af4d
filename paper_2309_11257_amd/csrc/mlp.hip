// Column surrogate: bfloat16 MLP on the MFMA units (C ABI in include/sg.h).
//
// GEMM: C[M][N] = A[M][K] B[K][N] with bfloat16 operands given by strides and
// float32 accumulation in v_mfma_f32_32x32x16_bf16.  A 256-thread workgroup
// computes a 128x128 tile; each of its four waves a 64x64 quarter as 2x2
// MFMA 32x32 tiles.  K advances in steps of 32 through LDS tiles held
// k-contiguous ([row][k], padded), so each lane's MFMA operand -- 8
// consecutive k of one row -- is one 16-byte LDS read.  Epilogues fuse bias,
// GELU (tanh form), GELU' and the bfloat16 conversion.  Weight gradients
// reduce over the batch with split-K partial tiles summed in a fixed order,
// so training is deterministic.
#include <math.h>
#include <string.h>

#include "../../include/sg.h"
#include "rt_internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

#define GBM 128
#define GBN 128
#define GBK 32
#define GPAD 8

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_DGELU = 3 };

struct GemmArgs {
    int M, N, K;
    const bf16 *A;
    int64_t am, ak;  // A(m, k) = A[m*am + k*ak]
    const bf16 *B;
    int64_t bk, bn;  // B(k, n) = B[k*bk + n*bn]
    float *C;        // EPI_F32 / EPI_BIAS output, [M][ldc]
    int64_t ldc;
    const float *bias;  // [N]
    float *Z;           // EPI_BIAS_GELU: pre-activation [M][ldc] (null: not kept)
    bf16 *H;            // EPI_BIAS_GELU: activation; EPI_DGELU: output dZ, [M][ldc]
    const float *Zp;    // EPI_DGELU: pre-activation of this layer's input [M][ldc]
    int ksplit;         // split-K chunks (grid.z); partials at C + z*M*ldc
};

// tanh(u) = 1 - 2 / (1 + exp(2u)): one exponential and one reciprocal
// (single-precision hardware approximations, far below the bfloat16 step of
// the activations); exp overflow gives 1, underflow -1
__device__ inline float tanh_e(float u)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * u));
}

__device__ inline float gelu_t(float z)
{
    const float c = 0.7978845608028654f;  // sqrt(2/pi)
    const float u = c * (z + 0.044715f * z * z * z);
    return 0.5f * z * (1.0f + tanh_e(u));
}

__device__ inline float dgelu_t(float z)
{
    const float c = 0.7978845608028654f;
    const float u = c * (z + 0.044715f * z * z * z);
    const float t = tanh_e(u);
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

// Staging of one 128 x GBK operand tile (rows = m or n, GBK consecutive k)
// from global memory: each thread moves GBK / 16 vectors of 8 bfloat16.  With the
// operand k-contiguous a vector is 8 consecutive k of one row; otherwise it is
// 8 consecutive rows at one k, transposed on the way into LDS.  Vectors that
// are not fully inside the matrix, or not 16-byte aligned, are assembled
// element by element (zero outside).
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

#define GNV (GBM * GBK / 8 / 256)

template <bool KCONT>
struct Stage {
    u16x8 v[GNV];
    __device__ inline void load(const bf16 *src, int64_t srow, int64_t sk, int row0, int nrows, int k0, int kend,
                                int tid)
    {
        const unsigned short *p = (const unsigned short *)src;
#pragma unroll
        for (int t = 0; t < GNV; t++) {
            const int vi = tid + 256 * t;
            int r, kk;
            if (KCONT) {
                r = vi / (GBK / 8);
                kk = (vi % (GBK / 8)) * 8;
            } else {
                kk = vi >> 4;
                r = (vi & 15) * 8;
            }
            const int gr = row0 + r, gk = k0 + kk;
            const int64_t off = (int64_t)gr * srow + (int64_t)gk * sk;
            const bool full = KCONT ? (gr < nrows && gk + 8 <= kend) : (gr + 8 <= nrows && gk < kend);
            if (full && ((((uintptr_t)(p + off)) & 15) == 0)) {
                v[t] = *(const u16x8 *)(p + off);
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int er = KCONT ? gr : gr + e, ek = KCONT ? gk + e : gk;
                    v[t][e] = (er < nrows && ek < kend) ? p[(int64_t)er * srow + (int64_t)ek * sk] : (unsigned short)0;
                }
            }
        }
    }
    __device__ inline void store(bf16 (*tile)[GBK + GPAD], int tid) const
    {
#pragma unroll
        for (int t = 0; t < GNV; t++) {
            const int vi = tid + 256 * t;
            if (KCONT) {
                *(u16x8 *)&tile[vi / (GBK / 8)][(vi % (GBK / 8)) * 8] = v[t];
            } else {
                const int kk = vi >> 4, r = (vi & 15) * 8;
#pragma unroll
                for (int e = 0; e < 8; e++) ((unsigned short *)&tile[r + e][0])[kk] = v[t][e];
            }
        }
    }
};

template <int EPI, bool KA, bool KB>
// three waves per SIMD: the accumulators live in the unified register file
__global__ __launch_bounds__(256, 3) void k_gemm(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) bf16 sA[GBM][GBK + GPAD];
    __shared__ __attribute__((aligned(16))) bf16 sB[GBN][GBK + GPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bm = blockIdx.x * GBM, bn = blockIdx.y * GBN;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // K range of this split
    const int kchunk = ((a.K + a.ksplit - 1) / a.ksplit + GBK - 1) / GBK * GBK;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(a.K, kbeg + kchunk);
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int q = 0; q < 16; q++) acc[i][j][q] = 0.0f;

    Stage<KA> ga;
    Stage<KB> gb;
    if (kbeg < kend) {
        ga.load(a.A, a.am, a.ak, bm, a.M, kbeg, kend, tid);
        gb.load(a.B, a.bn, a.bk, bn, a.N, kbeg, kend, tid);
    }
    for (int k0 = kbeg; k0 < kend; k0 += GBK) {
        __syncthreads();  // the previous tile has been consumed
        ga.store(sA, tid);
        gb.store(sB, tid);
        __syncthreads();
        if (k0 + GBK < kend) {  // next tile's loads in flight during the MFMAs
            ga.load(a.A, a.am, a.ak, bm, a.M, k0 + GBK, kend, tid);
            gb.load(a.B, a.bn, a.bk, bn, a.N, k0 + GBK, kend, tid);
        }
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            bf16x8 af[2], bfr[2];
            const int ko = kk + 8 * (lane >> 5);
#pragma unroll
            for (int i = 0; i < 2; i++) af[i] = *(const bf16x8 *)&sA[wm + i * 32 + (lane & 31)][ko];
#pragma unroll
            for (int j = 0; j < 2; j++) bfr[j] = *(const bf16x8 *)&sB[wn + j * 32 + (lane & 31)][ko];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    }
    // output element (row, col) of the 32x32 tile held in lane/item: column
    // and bias once per column block, one row base per row block and the
    // item's row step from a scalar product; bounds are tested only in the
    // tiles that cross the matrix edge
    const bool full = bm + GBM <= a.M && bn + GBN <= a.N;
    float *const Cz = (EPI == EPI_F32) ? a.C + (int64_t)blockIdx.z * a.M * a.ldc : a.C;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int col = bn + wn + j * 32 + (lane & 31);
        float bj = 0.0f;
        if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) bj = col < a.N ? a.bias[col] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const int r0 = bm + wm + i * 32 + 4 * (lane >> 5);
            const int64_t o0 = (int64_t)r0 * a.ldc + col;
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int dr = 8 * (q >> 2) + (q & 3);
                if (!full && (r0 + dr >= a.M || col >= a.N)) continue;
                const int64_t o = o0 + (int64_t)dr * a.ldc;
                const float v = acc[i][j][q];
                if (EPI == EPI_F32) {
                    Cz[o] = v;
                } else if (EPI == EPI_BIAS) {
                    a.C[o] = v + bj;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = v + bj;
                    if (a.Z) a.Z[o] = z;  // kept for the backward pass only
                    a.H[o] = (bf16)gelu_t(z);
                } else {  // EPI_DGELU
                    a.H[o] = (bf16)(v * dgelu_t(a.Zp[o]));
                }
            }
        }
    }
}

// sum of the split-K partials in chunk order
__global__ void k_sum_partials(const float *P, int64_t n, int S, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int z = 0; z < S; z++) s += P[(int64_t)z * n + i];
    out[i] = s;
}

// column sums (bias gradient) of a [M][N] bfloat16 matrix, first pass: chunk
// p of the rows (in order) per thread and column, partial sums to part[p][N];
// the partials are then added in chunk order (k_sum_partials)
#define COLSUM_CHUNKS 32
__global__ void k_colsum_bf16(const bf16 *D, int M, int N, float *part)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (c >= N) return;
    const int rows = (M + COLSUM_CHUNKS - 1) / COLSUM_CHUNKS;
    const int r0 = p * rows, r1 = min(M, r0 + rows);
    float s = 0.0f;
    for (int r = r0; r < r1; r++) s += (float)D[(int64_t)r * N + c];
    part[(int64_t)p * N + c] = s;
}

// loss gradient dY = 2 (Y - T) / (B n_out) in bfloat16, and per-block partial
// sums of (Y - T)^2
__global__ void k_mse(const float *Y, const float *T, int64_t n, float scale, bf16 *dY, float *part)
{
    __shared__ float sh[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e2 = 0.0f;
    if (i < n) {
        const float d = Y[i] - T[i];
        dY[i] = (bf16)(2.0f * d * scale);
        e2 = d * d;
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_to(const float *part, int64_t np, float scale, float *out)
{
    __shared__ float sh[256];
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < np; b += 256) s += part[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); bfloat16 copy of w
__global__ void k_adam(float *w, bf16 *wb, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = (bf16)wi;
}

__global__ void k_to_bf16(const float *w, bf16 *wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = (bf16)w[i];
}

// counter-based uniform in [-1, 1): splitmix64 of (seed, member, index)
__device__ inline uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// He-uniform weights (bound sqrt(6/fan_in)), zero biases
__global__ void k_init(float *w, int64_t n, int64_t wcount, float bound, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i < wcount) {
        const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)i));
        const float u = (float)((double)(r >> 11) * (1.0 / 9007199254740992.0)) * 2.0f - 1.0f;
        w[i] = bound * u;
    } else {
        w[i] = 0.0f;
    }
}

// gate: spread = sqrt(mean over outputs of the ensemble variance); trusted
// if spread <= tau and all features inside the training range
// gate: one wave per column; lanes take outputs and features round-robin,
// partial sums are combined by a fixed butterfly (deterministic)
__global__ __launch_bounds__(256) void k_gate(const float *Y, const float *X, const float *fmin, const float *fmax,
                                              int nm, int nc, int nout, int nin, float tau, float *spread,
                                              uint8_t *mask)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nc) return;  // whole wave
    double s2 = 0.0;
    for (int o = lane; o < nout; o += 64) {
        double mu = 0.0;
        for (int m = 0; m < nm; m++) mu += Y[((int64_t)m * nc + c) * nout + o];
        mu /= nm;
        double v = 0.0;
        for (int m = 0; m < nm; m++) {
            const double d = Y[((int64_t)m * nc + c) * nout + o] - mu;
            v += d * d;
        }
        s2 += nm > 1 ? v / (nm - 1) : 0.0;
    }
    int inside = 1;
    for (int f = lane; f < nin; f += 64) {
        const float x = X[(int64_t)c * nin + f];
        inside &= (x >= fmin[f] && x <= fmax[f]) ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s2 += __shfl_xor(s2, off, 64);
        inside &= __shfl_xor(inside, off, 64);
    }
    if (lane == 0) {
        const double sp = sqrt(s2 / nout);
        if (spread) spread[c] = (float)sp;
        mask[c] = (inside && sp <= (double)tau) ? 1 : 0;
    }
}

__global__ void k_standardize(const float *X, const float *mean, const float *std, const float *lg, int64_t n,
                              int nin, bf16 *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int f = (int)(i % nin);
    float x = X[i];
    if (lg[f] > 0.0f) x = log10f(fmaxf(x + lg[f], 1e-30f));
    out[i] = (bf16)((x - mean[f]) / std[f]);
}

// T[c][o] = (drag[o][c] - mean[o]) / std[o]: one thread per (c, o), o fastest
// so the writes are contiguous
__global__ void k_targets(const double *drag, const float *mean, const float *std, int nc, int nout, float *T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nc * nout) return;
    const int o = (int)(i % nout), c = (int)(i / nout);
    T[i] = (float)((drag[(int64_t)o * nc + c] - (double)mean[o]) / (double)std[o]);
}

// drag[o][c] <- ensemble mean of de-standardised outputs where mask[c]:
// a block takes 32 columns, reads their output rows contiguously and writes
// the drag rows contiguously, transposing through LDS
#define APPLY_COLS 32
__global__ __launch_bounds__(256) void k_apply_drag(const float *Y, const float *mean, const float *std,
                                                    const uint8_t *mask, int nm, int nc, int nout, double *drag)
{
    extern __shared__ double ap_tile[];  // [APPLY_COLS][nout]
    const int c0 = blockIdx.x * APPLY_COLS;
    const int ncols = min(APPLY_COLS, nc - c0);
    for (int e = threadIdx.x; e < ncols * nout; e += 256) {
        const int cl = e / nout, o = e % nout;
        double s = 0.0;
        if (mask[c0 + cl])
            for (int m = 0; m < nm; m++) s += (double)Y[((int64_t)m * nc + c0 + cl) * nout + o] * std[o] + mean[o];
        ap_tile[cl * nout + o] = s / nm;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ncols * nout; e += 256) {
        const int o = e / ncols, cl = e % ncols;
        if (mask[c0 + cl]) drag[(int64_t)o * nc + c0 + cl] = ap_tile[cl * nout + o];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layer {
    int in, out;
    int64_t woff, boff;  // offsets in the parameter vector
};

struct sg_net_s {
    sg_config cfg;
    hipStream_t stream;
    char err[256];
    int nl;  // total layers = n_layers + 1
    Layer L[16];
    int64_t P;  // parameters per member
    // per member: master w, bf16 copy, adam m, v, step
    float **w, **m, **v;
    bf16 **wb;
    int64_t *t;
    float *grad;  // [P]
    float *part;  // split-K partials / loss partials
    int64_t part_len;
    // activations for max_batch
    float **Z;  // [nl-1][B*hidden]
    bf16 **H;   // [nl-1]
    float *Yb;  // [B*n_out]
    bf16 *dY;   // [B*n_out]
    bf16 *dZ[2];
    void *allocs[64];
    int nallocs;
};

static void *net_alloc(sg_net n, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (n->nallocs >= 64) return nullptr;
    if (n->cfg.alloc)
        p = n->cfg.alloc(bytes, n->cfg.user);
    else if (hipMalloc(&p, bytes) != hipSuccess)
        p = nullptr;
    if (p) n->allocs[n->nallocs++] = p;
    return p;
}

static void net_release(sg_net n)
{
    for (int i = 0; i < n->nallocs; i++) {
        if (n->cfg.free)
            n->cfg.free(n->allocs[i], n->cfg.user);
        else if (!n->cfg.alloc)
            (void)hipFree(n->allocs[i]);
    }
    n->nallocs = 0;
    delete[] n->w;
    delete[] n->m;
    delete[] n->v;
    delete[] n->wb;
    delete[] n->t;
    delete[] n->Z;
    delete[] n->H;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

extern "C" rt_status sg_create(const sg_config *cfg, sg_net *out)
{
    if (!out) return RT_E_ARG;
    *out = nullptr;
    if (!cfg || cfg->n_members < 1 || cfg->n_in < 1 || cfg->n_hidden < 1 || cfg->n_layers < 1 || cfg->n_layers > 14 ||
        cfg->n_out < 1 || cfg->max_batch < 1)
        return RT_E_ARG;
    if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return RT_E_ARG;
    sg_net n = new sg_net_s();
    memset(n, 0, sizeof(*n));
    n->cfg = *cfg;
    n->stream = (hipStream_t)cfg->stream;
    n->nl = cfg->n_layers + 1;
    int64_t off = 0;
    for (int i = 0; i < n->nl; i++) {
        Layer &l = n->L[i];
        l.in = i == 0 ? cfg->n_in : cfg->n_hidden;
        l.out = i == n->nl - 1 ? cfg->n_out : cfg->n_hidden;
        l.woff = off;
        off += (int64_t)l.in * l.out;
    }
    for (int i = 0; i < n->nl; i++) {
        n->L[i].boff = off;
        off += n->L[i].out;
    }
    n->P = off;
    const int M = cfg->n_members;
    n->w = new float *[M];
    n->m = new float *[M];
    n->v = new float *[M];
    n->wb = new bf16 *[M];
    n->t = new int64_t[M];
    n->Z = new float *[n->nl];
    n->H = new bf16 *[n->nl];
    const int64_t B = cfg->max_batch, Hd = cfg->n_hidden;
    bool ok = true;
    for (int i = 0; i < M && ok; i++) {
        n->w[i] = (float *)net_alloc(n, sizeof(float) * n->P);
        n->m[i] = (float *)net_alloc(n, sizeof(float) * n->P);
        n->v[i] = (float *)net_alloc(n, sizeof(float) * n->P);
        n->wb[i] = (bf16 *)net_alloc(n, sizeof(bf16) * n->P);
        n->t[i] = 0;
        ok = n->w[i] && n->m[i] && n->v[i] && n->wb[i];
    }
    n->grad = (float *)net_alloc(n, sizeof(float) * n->P);
    // split-K partials for the largest weight gradient, and loss partials
    int64_t maxw = 0;
    for (int i = 0; i < n->nl; i++) maxw = maxw > (int64_t)n->L[i].in * n->L[i].out ? maxw : (int64_t)n->L[i].in * n->L[i].out;
    const int64_t maxo = cfg->n_hidden > cfg->n_out ? cfg->n_hidden : cfg->n_out;
    const int64_t front = 16 * maxw > COLSUM_CHUNKS * maxo ? 16 * maxw : COLSUM_CHUNKS * maxo;
    n->part_len = front + (B * cfg->n_out + 255) / 256 + 16;
    n->part = (float *)net_alloc(n, sizeof(float) * n->part_len);
    for (int i = 0; i < n->nl - 1 && ok; i++) {
        n->Z[i] = (float *)net_alloc(n, sizeof(float) * B * Hd);
        n->H[i] = (bf16 *)net_alloc(n, sizeof(bf16) * B * Hd);
        ok = n->Z[i] && n->H[i];
    }
    n->Yb = (float *)net_alloc(n, sizeof(float) * B * cfg->n_out);
    n->dY = (bf16 *)net_alloc(n, sizeof(bf16) * B * cfg->n_out);
    n->dZ[0] = (bf16 *)net_alloc(n, sizeof(bf16) * B * Hd);
    n->dZ[1] = (bf16 *)net_alloc(n, sizeof(bf16) * B * Hd);
    ok = ok && n->grad && n->part && n->Yb && n->dY && n->dZ[0] && n->dZ[1];
    if (!ok) {
        net_release(n);
        delete n;
        return RT_E_NOMEM;
    }
    for (int i = 0; i < M; i++) {
        for (int li = 0; li < n->nl; li++) {
            const Layer &l = n->L[li];
            const float bound = sqrtf(6.0f / (float)l.in);
            k_init<<<nblk((int64_t)l.in * l.out), 256, 0, n->stream>>>(
                n->w[i] + l.woff, (int64_t)l.in * l.out, (int64_t)l.in * l.out, bound,
                cfg->seed * 0x100000001b3ull + (uint64_t)i * 131 + (uint64_t)li);
        }
        (void)hipMemsetAsync(n->w[i] + n->L[0].boff, 0, sizeof(float) * (n->P - n->L[0].boff), n->stream);
        (void)hipMemsetAsync(n->m[i], 0, sizeof(float) * n->P, n->stream);
        (void)hipMemsetAsync(n->v[i], 0, sizeof(float) * n->P, n->stream);
        k_to_bf16<<<nblk(n->P), 256, 0, n->stream>>>(n->w[i], n->wb[i], n->P);
    }
    if (hipGetLastError() != hipSuccess) {
        net_release(n);
        delete n;
        return RT_E_DEVICE;
    }
    *out = n;
    return RT_OK;
}

extern "C" rt_status sg_destroy(sg_net n)
{
    if (!n) return RT_E_ARG;
    (void)hipStreamSynchronize(n->stream);
    net_release(n);
    delete n;
    return RT_OK;
}

extern "C" int64_t sg_param_count(sg_net n) { return n ? n->P : 0; }

extern "C" const char *sg_last_error(sg_net n) { return n ? n->err : "null net"; }

static rt_status sg_fail(sg_net n, rt_status s, const char *msg)
{
    if (n) snprintf(n->err, sizeof(n->err), "%s", msg);
    return s;
}

#define SG_HIP(call)                                               \
    do {                                                           \
        if ((call) != hipSuccess) return sg_fail(n, RT_E_DEVICE, #call); \
    } while (0)

extern "C" rt_status sg_get_params(sg_net n, int32_t member, float *params, int32_t where)
{
    if (!n || !params || member < 0 || member >= n->cfg.n_members) return RT_E_ARG;
    SG_HIP(hipMemcpyAsync(params, n->w[member], sizeof(float) * n->P,
                          where == RT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, n->stream));
    if (where == RT_HOST) SG_HIP(hipStreamSynchronize(n->stream));
    return RT_OK;
}

extern "C" rt_status sg_set_params(sg_net n, int32_t member, const float *params, int32_t where)
{
    if (!n || !params || member < 0 || member >= n->cfg.n_members) return RT_E_ARG;
    SG_HIP(hipMemcpyAsync(n->w[member], params, sizeof(float) * n->P,
                          where == RT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, n->stream));
    SG_HIP(hipMemsetAsync(n->m[member], 0, sizeof(float) * n->P, n->stream));
    SG_HIP(hipMemsetAsync(n->v[member], 0, sizeof(float) * n->P, n->stream));
    k_to_bf16<<<nblk(n->P), 256, 0, n->stream>>>(n->w[member], n->wb[member], n->P);
    n->t[member] = 0;
    if (where == RT_HOST) SG_HIP(hipStreamSynchronize(n->stream));
    return RT_OK;
}

// operand layouts picked at run time: A k-contiguous (ak == 1) or
// m-contiguous (am == 1), B k-contiguous (bk == 1) or n-contiguous (bn == 1)
template <int EPI>
static void gemm(const GemmArgs &a, hipStream_t s)
{
    dim3 grid((a.M + GBM - 1) / GBM, (a.N + GBN - 1) / GBN, a.ksplit);
    const bool ka = a.ak == 1, kb = a.bk == 1;
    if (ka && kb)
        k_gemm<EPI, true, true><<<grid, 256, 0, s>>>(a);
    else if (ka)
        k_gemm<EPI, true, false><<<grid, 256, 0, s>>>(a);
    else if (kb)
        k_gemm<EPI, false, true><<<grid, 256, 0, s>>>(a);
    else
        k_gemm<EPI, false, false><<<grid, 256, 0, s>>>(a);
}

// forward of one member for a batch of B; output to Yout [B][n_out]; the
// pre-activations are kept (for a backward pass) when keep_z
static void forward(sg_net n, int mem, const bf16 *X, float *Yout, int B, bool keep_z)
{
    const bf16 *in = X;
    for (int li = 0; li < n->nl; li++) {
        const Layer &l = n->L[li];
        GemmArgs a = {};
        a.M = B;
        a.N = l.out;
        a.K = l.in;
        a.A = in;
        a.am = l.in;
        a.ak = 1;
        a.B = n->wb[mem] + l.woff;  // W[out][in]: B(k, n) = W[n][k]
        a.bk = 1;
        a.bn = l.in;
        a.bias = n->w[mem] + l.boff;
        a.ldc = l.out;
        a.ksplit = 1;
        if (li < n->nl - 1) {
            a.Z = keep_z ? n->Z[li] : nullptr;
            a.H = n->H[li];
            gemm<EPI_BIAS_GELU>(a, n->stream);
            in = n->H[li];
        } else {
            a.C = Yout;
            gemm<EPI_BIAS>(a, n->stream);
        }
    }
}

extern "C" rt_status sg_forward(sg_net n, int32_t member, const uint16_t *X, float *Y, int32_t B)
{
    if (!n || !X || !Y || B < 1 || B > n->cfg.max_batch || member < -1 || member >= n->cfg.n_members)
        return sg_fail(n, RT_E_ARG, "bad sg_forward arguments");
    if (member >= 0) {
        forward(n, member, (const bf16 *)X, Y, B, false);
    } else {
        for (int m = 0; m < n->cfg.n_members; m++)
            forward(n, m, (const bf16 *)X, Y + (int64_t)m * B * n->cfg.n_out, B, false);
    }
    SG_HIP(hipGetLastError());
    return RT_OK;
}

// backward of one member after forward(); gradient into n->grad
static void backward(sg_net n, int mem, const bf16 *X, const float *T, int B, float *loss)
{
    const int nout = n->cfg.n_out;
    const int64_t ny = (int64_t)B * nout;
    const int64_t np = (ny + 255) / 256;
    float *lpart = n->part + n->part_len - np - 8;
    k_mse<<<(unsigned)np, 256, 0, n->stream>>>(n->Yb, T, ny, 1.0f / (float)ny, n->dY, lpart);
    if (loss) k_sum_to<<<1, 256, 0, n->stream>>>(lpart, np, 1.0f / (float)ny, loss);
    const bf16 *dcur = n->dY;  // gradient w.r.t. this layer's output (pre-activation for hidden layers)
    int which = 0;
    for (int li = n->nl - 1; li >= 0; li--) {
        const Layer &l = n->L[li];
        const bf16 *in = li == 0 ? X : n->H[li - 1];
        // dW[out][in] = sum_b d[b][out] * in[b][in]  (split-K over the batch)
        {
            GemmArgs a = {};
            a.M = l.out;
            a.N = l.in;
            a.K = B;
            a.A = dcur;  // A(m=out, k=b) = d[b][out]
            a.am = 1;
            a.ak = l.out;
            a.B = in;  // B(k=b, n=in) = in[b][in]
            a.bk = l.in;
            a.bn = 1;
            a.C = n->part;
            a.ldc = l.in;
            a.ksplit = B >= 2048 ? 16 : 1;
            gemm<EPI_F32>(a, n->stream);
            const int64_t nw = (int64_t)l.out * l.in;
            k_sum_partials<<<nblk(nw), 256, 0, n->stream>>>(n->part, nw, a.ksplit, n->grad + l.woff);
            k_colsum_bf16<<<dim3(nblk(l.out), COLSUM_CHUNKS), 256, 0, n->stream>>>(dcur, B, l.out, n->part);
            k_sum_partials<<<nblk(l.out), 256, 0, n->stream>>>(n->part, l.out, COLSUM_CHUNKS, n->grad + l.boff);
        }
        if (li > 0) {
            // d(in)[b][in] = sum_out d[b][out] W[out][in], times GELU'(Z_{li-1})
            GemmArgs a = {};
            a.M = B;
            a.N = l.in;
            a.K = l.out;
            a.A = dcur;  // A(m=b, k=out)
            a.am = l.out;
            a.ak = 1;
            a.B = n->wb[mem] + l.woff;  // B(k=out, n=in) = W[out][in]
            a.bk = l.in;
            a.bn = 1;
            a.ldc = l.in;
            a.Zp = n->Z[li - 1];
            a.H = n->dZ[which];
            a.ksplit = 1;
            gemm<EPI_DGELU>(a, n->stream);
            dcur = n->dZ[which];
            which ^= 1;
        }
    }
}

extern "C" rt_status sg_gradient(sg_net n, int32_t member, const uint16_t *X, const float *T, int32_t B, float *grads,
                                 int32_t where)
{
    if (!n || !X || !T || !grads || B < 1 || B > n->cfg.max_batch || member < 0 || member >= n->cfg.n_members)
        return sg_fail(n, RT_E_ARG, "bad sg_gradient arguments");
    forward(n, member, (const bf16 *)X, n->Yb, B, true);
    backward(n, member, (const bf16 *)X, T, B, nullptr);
    SG_HIP(hipMemcpyAsync(grads, n->grad, sizeof(float) * n->P,
                          where == RT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, n->stream));
    if (where == RT_HOST) SG_HIP(hipStreamSynchronize(n->stream));
    SG_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status sg_train_step(sg_net n, int32_t member, const uint16_t *X, const float *T, int32_t B, float lr,
                                   float *loss)
{
    if (!n || !X || !T || B < 1 || B > n->cfg.max_batch || member < 0 || member >= n->cfg.n_members)
        return sg_fail(n, RT_E_ARG, "bad sg_train_step arguments");
    forward(n, member, (const bf16 *)X, n->Yb, B, true);
    backward(n, member, (const bf16 *)X, T, B, loss);
    n->t[member] += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)n->t[member]));
    const float c2 = (float)(1.0 - pow(b2, (double)n->t[member]));
    k_adam<<<nblk(n->P), 256, 0, n->stream>>>(n->w[member], n->wb[member], n->m[member], n->v[member], n->grad, n->P,
                                               lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    SG_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status sg_gate(sg_net n, const float *Yens, const float *Xraw, const float *fmin, const float *fmax,
                             int32_t n_cols, float tau, float *spread, uint8_t *mask)
{
    if (!n || !Yens || !Xraw || !fmin || !fmax || !mask || n_cols < 0) return sg_fail(n, RT_E_ARG, "bad sg_gate arguments");
    if (n_cols == 0) return RT_OK;
    k_gate<<<(unsigned)((n_cols + 3) / 4), 256, 0, n->stream>>>(Yens, Xraw, fmin, fmax, n->cfg.n_members, n_cols,
                                                               n->cfg.n_out, n->cfg.n_in, tau, spread, mask);
    SG_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status sg_standardize(sg_net n, const float *Xraw, const float *mean, const float *std,
                                    const float *logfloor, int32_t n_cols, uint16_t *X)
{
    if (!n || !Xraw || !mean || !std || !logfloor || !X || n_cols < 0)
        return sg_fail(n, RT_E_ARG, "bad sg_standardize arguments");
    const int64_t tot = (int64_t)n_cols * n->cfg.n_in;
    if (tot == 0) return RT_OK;
    k_standardize<<<nblk(tot), 256, 0, n->stream>>>(Xraw, mean, std, logfloor, tot, n->cfg.n_in, (bf16 *)X);
    SG_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status sg_apply_drag(sg_net n, const float *Yens, const float *mean, const float *std,
                                   const uint8_t *mask, int32_t n_cols, int32_t nz, double *drag)
{
    if (!n || !Yens || !mean || !std || !mask || !drag || n_cols < 0)
        return sg_fail(n, RT_E_ARG, "bad sg_apply_drag arguments");
    if (nz < 1 || 2 * nz != n->cfg.n_out) return sg_fail(n, RT_E_ARG, "n_out must equal 2*nz");
    const int64_t tot = (int64_t)n_cols * n->cfg.n_out;
    if (tot == 0) return RT_OK;
    if ((size_t)APPLY_COLS * n->cfg.n_out * sizeof(double) > 65536) return sg_fail(n, RT_E_UNSUPPORTED, "n_out too large");
    k_apply_drag<<<(unsigned)((n_cols + APPLY_COLS - 1) / APPLY_COLS), 256,
                   (size_t)APPLY_COLS * n->cfg.n_out * sizeof(double), n->stream>>>(Yens, mean, std, mask,
                                                                                   n->cfg.n_members, n_cols,
                                                                                   n->cfg.n_out, drag);
    SG_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status sg_targets(sg_net n, const double *drag, const float *mean, const float *std, int32_t n_cols,
                                int32_t nz, float *T)
{
    if (!n || !drag || !mean || !std || !T || n_cols < 0) return sg_fail(n, RT_E_ARG, "bad sg_targets arguments");
    if (nz < 1 || 2 * nz != n->cfg.n_out) return sg_fail(n, RT_E_ARG, "n_out must equal 2*nz");
    const int64_t tot = (int64_t)n_cols * n->cfg.n_out;
    if (tot == 0) return RT_OK;
    k_targets<<<nblk(tot), 256, 0, n->stream>>>(drag, mean, std, n_cols, n->cfg.n_out, T);
    SG_HIP(hipGetLastError());
    return RT_OK;
}
