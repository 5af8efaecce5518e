// surrogate.hip -- MLP surrogate p(rates) on gfx950: BF16 operands, FP32
// accumulation on MFMA (v_mfma_f32_32x32x16_bf16), trained on the GPU.
//
// Network: 3 -> 256 -> 256 -> 1, ReLU hidden units, sigmoid output, inputs
// standardised log10 rate constants.  Numeric contract:
//   - matrix operands are BF16 (round to nearest even from FP32): the
//     standardised inputs xb, the weights W1b, W2b, W3b, the activations h1b,
//     h2b and the layer-2 error d2b;
//   - every product-sum accumulates in FP32; biases, losses, gradients and
//     the Adam state are FP32; FP32 master weights are rounded to BF16 after
//     every update;
//   - batch sums run in a fixed order (no atomics), so results are repeatable.
// Layer 2 (K = 256) and its two backward products run on MFMA; layers 1
// (K = 3) and 3 (N = 1) are vector work.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

constexpr int kH = 256;   // hidden width

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// C(m, n) = sum_k A(m, k) B(k, n) for BF16 A, B given by strides, FP32 C
// (row-major, ldc), optionally added to C.  M, N multiples of 32, K of 16;
// one wave per 32 x 32 tile of C.  Lane l holds row/column l % 32 and the
// k-slice 8 (l / 32) .. 8 (l / 32) + 7 of each 16-wide step for both
// operands; the 16 results of lane l are rows 8 (r / 4) + 4 (l / 32) + r % 4
// of column l % 32.
// ---------------------------------------------------------------------------
// An operand whose k-slices are contiguous (unit stride along k, 16-byte
// aligned rows) is read as one 16-byte load per lane; otherwise as eight
// 2-byte loads, which are coalesced across the 32 lanes of a half-wave when
// the other stride is 1.
template <bool kContig>
__device__ __forceinline__ bf16x8 load_slice(const uint16_t *p, long sk)
{
    bf16x8 v;
    if constexpr (kContig) {
        const uint4 w = *reinterpret_cast<const uint4 *>(p);
        v = __builtin_bit_cast(bf16x8, w);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = __builtin_bit_cast(__bf16, p[(long)e * sk]);
    }
    return v;
}

template <bool kAc, bool kBc>
__global__ __launch_bounds__(256) void gemm_bf16(const uint16_t *A, long sam, long sak, const uint16_t *B,
                                                 long sbk, long sbn, float *C, long ldc, int M, int N, int K,
                                                 int accumulate)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    const int tiles_n = N / 32;
    const int tm = wave / tiles_n, tn = wave % tiles_n;
    if (tm >= M / 32) return;
    const int rc = lane & 31, half = lane >> 5;
    const uint16_t *pa = A + (long)(tm * 32 + rc) * sam + (long)(8 * half) * sak;
    const uint16_t *pb = B + (long)(tn * 32 + rc) * sbn + (long)(8 * half) * sbk;
    floatx16 acc = {};
    // two 16-wide steps per trip, loads first, so both steps' loads are in
    // flight together; the MFMAs still run in ascending k
    int kb = 0;
    for (; kb + 32 <= K; kb += 32) {
        const bf16x8 a0 = load_slice<kAc>(pa + (long)kb * sak, sak);
        const bf16x8 b0 = load_slice<kBc>(pb + (long)kb * sbk, sbk);
        const bf16x8 a1 = load_slice<kAc>(pa + (long)(kb + 16) * sak, sak);
        const bf16x8 b1 = load_slice<kBc>(pb + (long)(kb + 16) * sbk, sbk);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
    }
    if (kb < K) {
        const bf16x8 a0 = load_slice<kAc>(pa + (long)kb * sak, sak);
        const bf16x8 b0 = load_slice<kBc>(pb + (long)kb * sbk, sbk);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const long row = tm * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        float *c = &C[row * ldc + tn * 32 + rc];
        *c = accumulate ? *c + acc[r] : acc[r];
    }
}

// The same product with k split over the four waves of a block, one 32 x 32
// tile per block: wave w runs the MFMA chain over k in [w K/4, (w+1) K/4),
// then the four partial tiles are added in wave order through LDS, so the
// result is repeatable.  For the small products of training (64-128 tiles)
// this gives four times the waves and a quarter of the dependent k-steps per
// wave.  K must be a multiple of 64; the grid is exactly one block per tile.
template <bool kAc, bool kBc>
__global__ __launch_bounds__(256) void gemm_bf16_splitk(const uint16_t *A, long sam, long sak, const uint16_t *B,
                                                        long sbk, long sbn, float *C, long ldc, int M, int N,
                                                        int K, int accumulate)
{
    __shared__ float part[4][16][64];
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const int tiles_n = N / 32;
    const int tm = (int)blockIdx.x / tiles_n, tn = (int)blockIdx.x % tiles_n;
    const int rc = lane & 31, half = lane >> 5;
    const int kq = K / 4;
    const long k0 = (long)w * kq;
    const uint16_t *pa = A + (long)(tm * 32 + rc) * sam + (k0 + 8 * half) * sak;
    const uint16_t *pb = B + (long)(tn * 32 + rc) * sbn + (k0 + 8 * half) * sbk;
    floatx16 acc = {};
    int kb = 0;
    for (; kb + 32 <= kq; kb += 32) {
        const bf16x8 a0 = load_slice<kAc>(pa + (long)kb * sak, sak);
        const bf16x8 b0 = load_slice<kBc>(pb + (long)kb * sbk, sbk);
        const bf16x8 a1 = load_slice<kAc>(pa + (long)(kb + 16) * sak, sak);
        const bf16x8 b1 = load_slice<kBc>(pb + (long)(kb + 16) * sbk, sbk);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
    }
    if (kb < kq) {
        const bf16x8 a0 = load_slice<kAc>(pa + (long)kb * sak, sak);
        const bf16x8 b0 = load_slice<kBc>(pb + (long)kb * sbk, sbk);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) part[w][r][lane] = acc[r];
    __syncthreads();
    // wave w finishes result registers 4w .. 4w + 3 of every lane
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * w + i;
        const float v = ((part[0][r][lane] + part[1][r][lane]) + part[2][r][lane]) + part[3][r][lane];
        const long row = tm * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        float *c = &C[row * ldc + tn * 32 + rc];
        *c = accumulate ? *c + v : v;
    }
}

// xb = bf16((x - mu) / sigma); pre1 = b1 + xb . W1b; h1b = bf16(relu(pre1)).
// One thread per (row, unit).
__global__ void layer1_forward(const float *x, int n, const float *mu, const float *sigma,
                               const uint16_t *W1b, const float *b1, uint16_t *xb, float *pre1,
                               uint16_t *h1b)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long row = t / kH;
    const int j = (int)(t % kH);
    if (row >= n) return;
    float acc = b1[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint16_t xk = to_bf16((x[row * 3 + k] - mu[k]) / sigma[k]);
        if (j == 0) xb[row * 3 + k] = xk;
        acc = fmaf(from_bf16(xk), from_bf16(W1b[j * 3 + k]), acc);
    }
    pre1[row * kH + j] = acc;
    h1b[row * kH + j] = to_bf16(acc > 0.0f ? acc : 0.0f);
}

// pre2 += b2 (pre2 holds the product); h2b = bf16(relu(pre2)).
__global__ void layer2_epilogue(float *pre2, int n, const float *b2, uint16_t *h2b)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n * kH) return;
    const float v = pre2[t] + b2[t % kH];
    pre2[t] = v;
    h2b[t] = to_bf16(v > 0.0f ? v : 0.0f);
}

// Per row: z = b3 + sum_j h2b W3b (j in order), p = sigmoid(z), weighted
// binary cross-entropy against the soft target y, dz = w (p - y) / sum w.
__global__ void layer3_forward_loss(const uint16_t *h2b, int n, const uint16_t *W3b, const float *b3,
                                    const float *y, const float *w, float inv_wsum, float *p_out,
                                    float *loss_row, float *dz)
{
    const int row = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (row >= n) return;
    float z = b3[0];
    for (int j = 0; j < kH; ++j) z = fmaf(from_bf16(h2b[(long)row * kH + j]), from_bf16(W3b[j]), z);
    const float p = 1.0f / (1.0f + expf(-z));
    if (p_out) p_out[row] = p;
    if (y) {
        const float yy = y[row], ww = w[row];
        // log(1 + e^-|z|) + max(z, 0) - z y  (stable form of the cross-entropy)
        const float l = fmaxf(z, 0.0f) - z * yy + log1pf(expf(-fabsf(z)));
        loss_row[row] = ww * l * inv_wsum;
        dz[row] = ww * (p - yy) * inv_wsum;
    }
}

// Batch reductions (column sums over the n rows of a [n][256] activation):
// a block of 16 columns x 64 row slices; thread (c, q) accumulates rows q,
// q + 64, q + 128, ... of column c in order (a wave reads 16 consecutive
// columns of 4 rows, 64 bytes each), then the 64 slice sums are added in
// slice order, so the result does not depend on scheduling.  16 blocks for
// the 256 columns keep the rows per thread short: with n = 512 the reduction
// is latency bound, not bandwidth bound.
constexpr int kColBlock = 16;
constexpr int kSlices = 64;

// dW3[j] = sum_b dz_b h2b[b][j], db3 = sum_b dz_b; d2 = dz W3b relu'(pre2)
// stored as d2b = bf16(d2) (the operand of both layer-2 backward products);
// db2[j] = sum_b d2[b][j] (FP32, before rounding).
__global__ __launch_bounds__(kColBlock * kSlices) void layer3_backward(
    const uint16_t *h2b, const float *pre2, int n, const uint16_t *W3b, const float *dz, float *dW3,
    float *db3, float *db2, uint16_t *d2b)
{
    __shared__ float red[3][kSlices][kColBlock];
    const int c = (int)(threadIdx.x % kColBlock), q = (int)(threadIdx.x / kColBlock);
    const int j = (int)blockIdx.x * kColBlock + c;
    const float w3 = from_bf16(W3b[j]);
    float sw = 0.0f, sd = 0.0f, sz = 0.0f;
    for (int b = q; b < n; b += kSlices) {
        const long t = (long)b * kH + j;
        const float g = dz[b];
        sw = fmaf(g, from_bf16(h2b[t]), sw);
        sz += g;
        const float d = pre2[t] > 0.0f ? g * w3 : 0.0f;
        sd += d;
        d2b[t] = to_bf16(d);
    }
    red[0][q][c] = sw;
    red[1][q][c] = sd;
    red[2][q][c] = sz;
    __syncthreads();
    if (q == 0) {
        float a = 0.0f, bb = 0.0f, z = 0.0f;
        for (int r = 0; r < kSlices; ++r) {
            a += red[0][r][c];
            bb += red[1][r][c];
            z += red[2][r][c];
        }
        dW3[j] = a;
        db2[j] = bb;
        if (j == 0) db3[0] = z;
    }
}

// d1 = dh1 relu'(pre1); dW1[j][k] = sum_b d1 xb[b][k]; db1[j] = sum_b d1.
__global__ __launch_bounds__(kColBlock * kSlices) void layer1_backward(
    const float *dh1, const float *pre1, const uint16_t *xb, int n, float *dW1, float *db1)
{
    __shared__ float red[4][kSlices][kColBlock];
    const int c = (int)(threadIdx.x % kColBlock), q = (int)(threadIdx.x / kColBlock);
    const int j = (int)blockIdx.x * kColBlock + c;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, sb = 0.0f;
    for (int b = q; b < n; b += kSlices) {
        const long t = (long)b * kH + j;
        const float d = pre1[t] > 0.0f ? dh1[t] : 0.0f;
        s0 = fmaf(d, from_bf16(xb[b * 3 + 0]), s0);
        s1 = fmaf(d, from_bf16(xb[b * 3 + 1]), s1);
        s2 = fmaf(d, from_bf16(xb[b * 3 + 2]), s2);
        sb += d;
    }
    red[0][q][c] = s0;
    red[1][q][c] = s1;
    red[2][q][c] = s2;
    red[3][q][c] = sb;
    __syncthreads();
    if (q == 0) {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, ab = 0.0f;
        for (int r = 0; r < kSlices; ++r) {
            a0 += red[0][r][c];
            a1 += red[1][r][c];
            a2 += red[2][r][c];
            ab += red[3][r][c];
        }
        dW1[j * 3 + 0] = a0;
        dW1[j * 3 + 1] = a1;
        dW1[j * 3 + 2] = a2;
        db1[j] = ab;
    }
}

// out[0] = sum of the n per-row losses: thread t sums rows t, t + 256, ...
// in order (FP64), then the 256 partial sums are added in thread order.
__global__ __launch_bounds__(256) void loss_sum(const float *loss_row, int n, float *out)
{
    __shared__ double part[256];
    const int t = (int)threadIdx.x;
    double acc = 0.0;
    for (int b = t; b < n; b += 256) acc += (double)loss_row[b];
    part[t] = acc;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int r = 0; r < 256; ++r) s += part[r];
        out[0] = (float)s;
    }
}

// Adam on FP32 masters; BF16 copies of the weight matrices refreshed.
__global__ void adam_update(float *w, const float *g, float *m, float *v, uint16_t *wb, long count,
                            float lr, float beta1, float beta2, float eps, float bc1, float bc2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
}

__global__ void round_bf16(const float *w, uint16_t *wb, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) wb[i] = to_bf16(w[i]);
}

// ---------------------------------------------------------------------------
// Inference + gate: 32 points per block of 256 threads.  Layer 1 into LDS as
// BF16, layer 2 on MFMA (wave w owns output columns 64 w .. 64 w + 63), layer
// 3 products staged in LDS and summed per point in column order.  A point
// uses the surrogate when it lies in the training hull (n.x <= d for every
// facet, in log10-rate space) and |p - threshold| >= margin.
// ---------------------------------------------------------------------------
// Hull test of a tile's 32 points, spread over the block's 256 threads: thread
// t tests point t % 32 against facets t / 32, t / 32 + 8, ...  A point found
// outside any facet (n.x > d + tol) has its flag cleared; the flags start at 1.
__device__ __forceinline__ void hull_test(const float *xs, const float *planes, int n_planes, float hull_tol,
                                          int *inside_s)
{
    const int tid = (int)threadIdx.x;
    const int r = tid & 31;
    const float a0 = xs[r * 3], a1 = xs[r * 3 + 1], a2 = xs[r * 3 + 2];
    bool ok = true;
    for (int f = tid >> 5; f < n_planes && ok; f += 8) {
        const float *pl = planes + 4 * f;
        const float v = pl[0] * a0 + pl[1] * a1 + pl[2] * a2;
        ok = v <= pl[3] + hull_tol;
    }
    if (!ok) inside_s[r] = 0;
}

__global__ __launch_bounds__(256) void mlp_query(const float *x, long n, const float *mu,
                                                 const float *sigma, const uint16_t *W1b,
                                                 const float *b1, const uint16_t *W2b,
                                                 const float *b2, const uint16_t *W3b,
                                                 const float *b3, const float *planes, int n_planes,
                                                 float hull_tol, float threshold, float margin,
                                                 float *p_out, uint8_t *use)
{
    __shared__ uint16_t h1s[32 * kH];
    __shared__ float prod[32 * kH];
    __shared__ float xs[32 * 3], xn[32 * 3];
    __shared__ int inside_s[32];
    const int tid = (int)threadIdx.x;
    const long base = (long)blockIdx.x * 32;
    if (tid < 96) {
        const long row = base + tid / 3;
        const int c = tid % 3;
        const float v = row < n ? x[row * 3 + c] : 0.0f;
        xs[tid] = v;
        xn[tid] = from_bf16(to_bf16((v - mu[c]) / sigma[c]));   // once per input, not per unit
    }
    if (tid < 32) inside_s[tid] = 1;
    __syncthreads();
    {
        const int j = tid;
        float w0 = from_bf16(W1b[j * 3]), w1 = from_bf16(W1b[j * 3 + 1]), w2 = from_bf16(W1b[j * 3 + 2]);
        const float bj = b1[j];
        for (int r = 0; r < 32; ++r) {
            float acc = bj;
            acc = fmaf(xn[r * 3 + 0], w0, acc);
            acc = fmaf(xn[r * 3 + 1], w1, acc);
            acc = fmaf(xn[r * 3 + 2], w2, acc);
            h1s[r * kH + j] = to_bf16(acc > 0.0f ? acc : 0.0f);
        }
    }
    if (use) hull_test(xs, planes, n_planes, hull_tol, inside_s);
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int rc = lane & 31, half = lane >> 5;
#pragma unroll
    for (int tile = 0; tile < 2; ++tile) {
        const int col = wave * 64 + tile * 32 + rc;   // output unit of this lane
        floatx16 acc = {};
        for (int kb = 0; kb < kH; kb += 16) {
            bf16x8 a, b;
            const int k0 = kb + 8 * half;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = __builtin_bit_cast(__bf16, h1s[rc * kH + k0 + e]);
                b[e] = __builtin_bit_cast(__bf16, W2b[(long)col * kH + k0 + e]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        const float b2c = b2[col];
        const float w3 = from_bf16(W3b[col]);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r / 4) + 4 * half + (r % 4);
            const float v = acc[r] + b2c;
            prod[row * kH + col] = from_bf16(to_bf16(v > 0.0f ? v : 0.0f)) * w3;
        }
    }
    __syncthreads();
    if (tid < 32) {
        const long row = base + tid;
        float z = b3[0];
        for (int j = 0; j < kH; ++j) z += prod[tid * kH + j];
        const float p = 1.0f / (1.0f + expf(-z));
        if (row < n) {
            p_out[row] = p;
            if (use) {
                const bool inside = n_planes > 0 && inside_s[tid] != 0;
                use[row] = (inside && fabsf(p - threshold) >= margin) ? 1 : 0;
            }
        }
    }
}

// LDS rows (a column of W2) are padded by 8 bfloat16 values, so that the
// 16-byte operand reads of the 32 lanes of a half-wave (one row each) start
// on different banks instead of all on the same one.
constexpr int kQRow = kH + 8;

// ---------------------------------------------------------------------------
// Inference + gate, one tile of 32 points per wave: each block (eight waves,
// two per SIMD, so that one wave's vector work overlaps the other's matrix
// work) stages W2 in LDS once; every wave then runs its own tiles from start
// to end, with no block barrier after the staging.  Per tile:
//  - layer 1 on the matrix cores, 32 hidden units at a time: one
//    v_mfma_f32_32x32x16_bf16 of the units' rows (w0, w1, w2 and b1 split
//    into three bfloat16 parts that add up to it, from LDS) by the tile's
//    inputs (n0, n1, n2, 1, 1, 1); the inputs and weights are bfloat16
//    values, so every product is exact and the sum is accumulated in FP32.
//    Lane l then holds units 8 (r / 4) + 4 (l / 32) + r % 4 (r = 0 .. 15) of
//    the block for point l % 32: after ReLU and rounding, the A operands of
//    the block's two layer-2 steps, in an order of k that W2's staging
//    follows (within every 16 k, the second and third groups of four trade
//    places), so that no value moves between lanes;
//  - layer 2: v_mfma_f32_32x32x16_bf16 adds each step to the eight 32-column
//    groups' accumulators (B from LDS);
//  - layer 3: every lane adds its columns' contributions to its 16 rows, then
//    the 32 lanes of each half sum by shuffles;
//  - the hull test spread over the two lanes of each point.
// Same numeric contract and gate as the other query kernels.
// ---------------------------------------------------------------------------
// f rounded to bfloat16 (nearest, ties to even) and back, by the hardware
// conversion (the same value as to_bf16 for finite f).
__device__ __forceinline__ float rne_bf16(float f) { return (float)(__bf16)f; }

// A lane's value moved across its 16-lane row by the DPP control ctrl.
template <int ctrl>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
}

constexpr int kQueryWaves = 8;
constexpr size_t kWaveQueryLds = (size_t)kH * kQRow * 2 + (size_t)kH * 16;
constexpr int kLdsPlanes = 1280;   // hull facets staged in LDS (a hull of n points has at most 2n - 4)

__global__ __launch_bounds__(64 * kQueryWaves) void mlp_query_waves(
    const float *x, long n, const float *mu, const float *sigma, const uint16_t *W1b, const float *b1,
    const uint16_t *W2b, const float *b2, const uint16_t *W3b, const float *b3, const float *planes, int n_planes,
    int n_lds_planes, float hull_tol, float threshold, float margin, float *p_out, uint8_t *use)
{
    extern __shared__ uint16_t qsm[];
    uint16_t *W2s = qsm;                                                // [col][k'] (row stride kQRow)
    uint4 *W1s = reinterpret_cast<uint4 *>(W2s + kH * kQRow);           // [unit]: layer 1's A row
    float4 *Ps = reinterpret_cast<float4 *>(W1s + kH);                  // facets 0 .. n_lds_planes - 1
    const int tid = (int)threadIdx.x;
    {
        // W2 by groups of four k: within every 16, groups 1 and 2 trade places
        const uint2 *src = reinterpret_cast<const uint2 *>(W2b);
        uint2 *dst = reinterpret_cast<uint2 *>(W2s);
        for (int i = tid; i < kH * kH / 4; i += 64 * kQueryWaves) {
            const int c = i % (kH / 4), q = c & 3;
            const int cd = (c & ~3) | (q == 1 ? 2 : q == 2 ? 1 : q);
            dst[(i / (kH / 4)) * (kQRow / 4) + cd] = src[i];
        }
        if (tid < kH) {
            // b1 = hi + lo + lo2, each a bfloat16 value (the two differences
            // are exact in FP32)
            const float b = b1[tid];
            const __bf16 hi = (__bf16)b;
            const float r1 = b - (float)hi;
            const __bf16 lo = (__bf16)r1;
            const __bf16 lo2 = (__bf16)(r1 - (float)lo);
            bf16x8 a;
            a[0] = __builtin_bit_cast(__bf16, W1b[tid * 3]);
            a[1] = __builtin_bit_cast(__bf16, W1b[tid * 3 + 1]);
            a[2] = __builtin_bit_cast(__bf16, W1b[tid * 3 + 2]);
            a[3] = hi;
            a[4] = lo;
            a[5] = lo2;
            a[6] = (__bf16)0.0f;
            a[7] = (__bf16)0.0f;
            W1s[tid] = __builtin_bit_cast(uint4, a);
            // b2 the same way, in the padding of column tid's W2 row (k' = 256 ..
            // 263), for one more layer-2 step against the constant input 1
            const float c = b2[tid];
            const __bf16 chi = (__bf16)c;
            const float c1 = c - (float)chi;
            const __bf16 clo = (__bf16)c1;
            const __bf16 clo2 = (__bf16)(c1 - (float)clo);
            bf16x8 bb;
            bb[0] = chi;
            bb[1] = clo;
            bb[2] = clo2;
            for (int e = 3; e < 8; ++e) bb[e] = (__bf16)0.0f;
            *reinterpret_cast<uint4 *>(W2s + tid * kQRow + kH) = __builtin_bit_cast(uint4, bb);
        }
        // facets with the tolerance added to their offsets once
        for (int f = tid; f < n_lds_planes; f += 64 * kQueryWaves)
            Ps[f] = make_float4(planes[4 * f], planes[4 * f + 1], planes[4 * f + 2], planes[4 * f + 3] + hull_tol);
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int rc = lane & 31, half = lane >> 5;
    const float bias3 = b3[0];
    const float mu0 = mu[0], mu1 = mu[1], mu2 = mu[2], sg0 = sigma[0], sg1 = sigma[1], sg2 = sigma[2];
    const long n_tiles = (n + 31) / 32;
    const long stride = (long)gridDim.x * kQueryWaves;
    // this lane's point of the wave's next tile, loaded one tile ahead
    long tile = (long)blockIdx.x * kQueryWaves + wave;
    float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
    if (tile * 32 + rc < n) {
        y0 = x[(tile * 32 + rc) * 3];
        y1 = x[(tile * 32 + rc) * 3 + 1];
        y2 = x[(tile * 32 + rc) * 3 + 2];
    }
    for (; tile < n_tiles; tile += stride) {
        const long row = tile * 32 + rc;   // this lane's point (both halves hold it)
        const float x0 = y0, x1 = y1, x2 = y2;
        const long nrow = (tile + stride) * 32 + rc;
        if (nrow < n) {
            y0 = x[nrow * 3];
            y1 = x[nrow * 3 + 1];
            y2 = x[nrow * 3 + 2];
        }
        const float n0 = rne_bf16((x0 - mu0) / sg0);
        const float n1 = rne_bf16((x1 - mu1) / sg1);
        const float n2 = rne_bf16((x2 - mu2) / sg2);
        // layer 1's B operand: this point's inputs at k = 0 .. 5 (half 0);
        // k = 8 .. 15 (half 1) are 0, as are the A rows there
        bf16x8 xin;
        xin[0] = (__bf16)(half ? 0.0f : n0);
        xin[1] = (__bf16)(half ? 0.0f : n1);
        xin[2] = (__bf16)(half ? 0.0f : n2);
        xin[3] = (__bf16)(half ? 0.0f : 1.0f);
        xin[4] = xin[3];
        xin[5] = xin[3];
        xin[6] = (__bf16)0.0f;
        xin[7] = (__bf16)0.0f;
        floatx16 acc[8];
        // units 32 bk .. 32 bk + 31 for the tile's 32 points, and the two
        // layer-2 steps they feed
        auto block = [&](int bk) {
            const uint4 wr = W1s[32 * bk + rc];
            const bf16x8 w = __builtin_bit_cast(bf16x8, half ? make_uint4(0u, 0u, 0u, 0u) : wr);
            const floatx16 h1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, xin, floatx16{}, 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                bf16x8 a;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    // ReLU as an integer max of the bit pattern (the same
                    // value as max(h, 0) for every h that is not a NaN), then
                    // v_cvt_pk_bf16_f32: round to nearest even
                    const int hb = __float_as_int(h1[8 * t + e]);
                    a[e] = (__bf16)__int_as_float(hb > 0 ? hb : 0);
                }
                const uint16_t *bcol = W2s + rc * kQRow + 8 * half + 16 * (2 * bk + t);
#pragma unroll
                for (int g = 0; g < 8; ++g) {
                    const bf16x8 b =
                        __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(bcol + g * 32 * kQRow));
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[g], 0, 0, 0);
                }
            }
        };
        {
            // the accumulators start with the layer-2 bias: inputs (1, 1, 1)
            // against each column's three parts (half 1 holds zeros, so what
            // its B operand reads past the padding does not count)
            bf16x8 one;
#pragma unroll
            for (int e = 0; e < 8; ++e) one[e] = (__bf16)(half == 0 && e < 3 ? 1.0f : 0.0f);
            const uint16_t *bpad = W2s + rc * kQRow + kH + 8 * half;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(bpad + g * 32 * kQRow));
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(one, b, floatx16{}, 0, 0, 0);
            }
        }
#pragma unroll 1
        for (int bk = 0; bk < 8; ++bk) block(bk);
        // layer 3: rows 8 (r / 4) + 4 half + r % 4 of column 32 g + rc (bias
        // included), two column groups at a time: the two rounded activations
        // and their weights as bfloat16 pairs, one v_dot2_f32_bf16 (exact
        // products, FP32 sum) per row
        float zr[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) zr[r] = 0.0f;
#pragma unroll
        for (int g = 0; g < 8; g += 2) {
            bf16x2 w;
            w[0] = __builtin_bit_cast(__bf16, W3b[g * 32 + rc]);
            w[1] = __builtin_bit_cast(__bf16, W3b[(g + 1) * 32 + rc]);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // ReLU as an integer max of the bit pattern, as in layer 1
                const int v0 = __float_as_int(acc[g][r]), v1 = __float_as_int(acc[g + 1][r]);
                bf16x2 h;
                h[0] = (__bf16)__int_as_float(v0 > 0 ? v0 : 0);
                h[1] = (__bf16)__int_as_float(v1 > 0 ? v1 : 0);
                zr[r] = __builtin_amdgcn_fdot2_f32_bf16(h, w, zr[r], false);
            }
        }
        // sum over the 32 columns of each half: then every lane of half h
        // holds the sums of rows 8 (r / 4) + 4 h + r % 4.  Within each 16-lane
        // row by DPP moves (swap neighbours, swap pairs, mirror the 8-lane
        // halves, mirror the row), then across the two rows of the half.
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float v = zr[r];
            v += dpp_f32<0xB1>(v);    // quad_perm [1, 0, 3, 2]
            v += dpp_f32<0x4E>(v);    // quad_perm [2, 3, 0, 1]
            v += dpp_f32<0x141>(v);   // row_half_mirror
            v += dpp_f32<0x140>(v);   // row_mirror
            zr[r] = v + __shfl_xor(v, 16, 64);
        }
        // row rc's sum is held by the half whose rows include it
        const int idx = 4 * (rc >> 3) + (rc & 3);
        float mine = zr[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mine = idx == r ? zr[r] : mine;
        const float z = bias3 + __shfl(mine, ((rc >> 2) & 1) * 32 + rc, 64);
        // hull: the two lanes of a point take alternate facets (from LDS, the
        // lanes of a half reading one facet at a time), without early exit
        bool ok = true;
        {
            int f = half;
#pragma unroll 4
            for (; f < n_lds_planes; f += 2) {
                const float4 pl = Ps[f];
                const float v = pl.x * x0 + pl.y * x1 + pl.z * x2;
                ok = ok && (v <= pl.w);
            }
            for (; f < n_planes; f += 2) {
                const float *pl = planes + 4 * f;
                const float v = pl[0] * x0 + pl[1] * x1 + pl[2] * x2;
                ok = ok && (v <= pl[3] + hull_tol);
            }
        }
        // (the shuffle runs on every lane: the partner's value must be written)
        const int other = __shfl(ok ? 1 : 0, lane ^ 32, 64);
        const bool inside = n_planes > 0 && ok && other != 0;
        if (half == 0 && row < n) {
            const float p = 1.0f / (1.0f + expf(-z));
            p_out[row] = p;
            if (use) use[row] = (inside && fabsf(p - threshold) >= margin) ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers.
// ---------------------------------------------------------------------------
static unsigned blocks_for(long n, int threads) { return (unsigned)((n + threads - 1) / threads); }

hipError_t sg_gemm(hipStream_t s, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk,
                   long sbn, float *C, long ldc, int M, int N, int K, int accumulate)
{
    const long waves = (long)(M / 32) * (N / 32);
    // unit stride along k, and every lane's first element 16-byte aligned
    // (k offsets are multiples of 8 elements)
    auto contig = [](const uint16_t *p, long sk, long so) {
        return sk == 1 && so % 8 == 0 && (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
    };
    const bool ac = contig(A, sak, sam), bc = contig(B, sbk, sbn);
    if (K % 64 == 0 && waves <= 1024) {
        // few tiles: split k over the four waves of a block, one block per tile
        const dim3 tgrid((unsigned)waves), tblock(256);
        if (ac && bc)
            hipLaunchKernelGGL((gemm_bf16_splitk<true, true>), tgrid, tblock, 0, s, A, sam, sak, B, sbk, sbn, C,
                               ldc, M, N, K, accumulate);
        else if (ac)
            hipLaunchKernelGGL((gemm_bf16_splitk<true, false>), tgrid, tblock, 0, s, A, sam, sak, B, sbk, sbn, C,
                               ldc, M, N, K, accumulate);
        else if (bc)
            hipLaunchKernelGGL((gemm_bf16_splitk<false, true>), tgrid, tblock, 0, s, A, sam, sak, B, sbk, sbn, C,
                               ldc, M, N, K, accumulate);
        else
            hipLaunchKernelGGL((gemm_bf16_splitk<false, false>), tgrid, tblock, 0, s, A, sam, sak, B, sbk, sbn,
                               C, ldc, M, N, K, accumulate);
        return hipGetLastError();
    }
    const dim3 grid(blocks_for(waves, 4)), block(256);
    if (ac && bc)
        hipLaunchKernelGGL((gemm_bf16<true, true>), grid, block, 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N,
                           K, accumulate);
    else if (ac)
        hipLaunchKernelGGL((gemm_bf16<true, false>), grid, block, 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M,
                           N, K, accumulate);
    else if (bc)
        hipLaunchKernelGGL((gemm_bf16<false, true>), grid, block, 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M,
                           N, K, accumulate);
    else
        hipLaunchKernelGGL((gemm_bf16<false, false>), grid, block, 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M,
                           N, K, accumulate);
    return hipGetLastError();
}

hipError_t sg_layer1_forward(hipStream_t s, const float *x, int n, const float *mu, const float *sigma,
                             const uint16_t *W1b, const float *b1, uint16_t *xb, float *pre1, uint16_t *h1b)
{
    hipLaunchKernelGGL(layer1_forward, dim3(blocks_for((long)n * kH, 256)), dim3(256), 0, s, x, n, mu,
                       sigma, W1b, b1, xb, pre1, h1b);
    return hipGetLastError();
}

hipError_t sg_layer2_epilogue(hipStream_t s, float *pre2, int n, const float *b2, uint16_t *h2b)
{
    hipLaunchKernelGGL(layer2_epilogue, dim3(blocks_for((long)n * kH, 256)), dim3(256), 0, s, pre2, n, b2, h2b);
    return hipGetLastError();
}

hipError_t sg_layer3_forward_loss(hipStream_t s, const uint16_t *h2b, int n, const uint16_t *W3b,
                                  const float *b3, const float *y, const float *w, float inv_wsum,
                                  float *p_out, float *loss_row, float *dz)
{
    hipLaunchKernelGGL(layer3_forward_loss, dim3(blocks_for(n, 256)), dim3(256), 0, s, h2b, n, W3b, b3, y, w,
                       inv_wsum, p_out, loss_row, dz);
    return hipGetLastError();
}

hipError_t sg_layer3_backward(hipStream_t s, const uint16_t *h2b, const float *pre2, int n,
                              const uint16_t *W3b, const float *dz, float *dW3, float *db3, float *db2,
                              uint16_t *d2b)
{
    hipLaunchKernelGGL(layer3_backward, dim3(kH / kColBlock), dim3(kColBlock * kSlices), 0, s, h2b, pre2, n,
                       W3b, dz, dW3, db3, db2, d2b);
    return hipGetLastError();
}

hipError_t sg_layer1_backward(hipStream_t s, const float *dh1, const float *pre1, const uint16_t *xb, int n,
                              float *dW1, float *db1)
{
    hipLaunchKernelGGL(layer1_backward, dim3(kH / kColBlock), dim3(kColBlock * kSlices), 0, s, dh1, pre1, xb,
                       n, dW1, db1);
    return hipGetLastError();
}

hipError_t sg_loss_sum(hipStream_t s, const float *loss_row, int n, float *out)
{
    hipLaunchKernelGGL(loss_sum, dim3(1), dim3(256), 0, s, loss_row, n, out);
    return hipGetLastError();
}

hipError_t sg_adam(hipStream_t s, float *w, const float *g, float *m, float *v, uint16_t *wb, long count,
                   float lr, float beta1, float beta2, float eps, float bc1, float bc2)
{
    hipLaunchKernelGGL(adam_update, dim3(blocks_for(count, 256)), dim3(256), 0, s, w, g, m, v, wb, count, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t sg_round(hipStream_t s, const float *w, uint16_t *wb, long count)
{
    hipLaunchKernelGGL(round_bf16, dim3(blocks_for(count, 256)), dim3(256), 0, s, w, wb, count);
    return hipGetLastError();
}

// The neighbourhood gate: the six points x +- delta e_k of every query point
// (log10 rate constants), and the test that the network's output at each of
// them lies on the same side of the threshold as at the point itself, at
// least `margin` away from it.
__global__ void expand_neighbours(const float *x, long n, float delta, float *x6)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * n) return;
    const long pnt = i / 6;
    const int k = (int)(i % 6);
    const int axis = k >> 1;
    const float step = (k & 1) ? -delta : delta;
#pragma unroll
    for (int a = 0; a < 3; ++a) x6[3 * i + a] = x[3 * pnt + a] + (a == axis ? step : 0.0f);
}

__global__ void neighbour_gate(const float *p, const float *p6, long n, float threshold, float margin, uint8_t *use)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !use[i]) return;
    const float side = p[i] >= threshold ? 1.0f : -1.0f;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) ok = ok && (p6[6 * i + k] - threshold) * side >= margin;
    use[i] = ok ? 1 : 0;
}

hipError_t sg_expand_neighbours(hipStream_t s, const float *x, long n, float delta, float *x6)
{
    hipLaunchKernelGGL(expand_neighbours, dim3(blocks_for(6 * n, 256)), dim3(256), 0, s, x, n, delta, x6);
    return hipGetLastError();
}

// Confirmation of answered points by a few SMC trajectories each: an answer
// on the FALSE side stands only if none of its trials satisfied the formula,
// one on the TRUE side only if all of them did (an entry with more successes
// than trials withdraws its answer).
__global__ void confirm_answers(const float *p, const unsigned long long *succ, const unsigned long long *trials,
                                long n, float threshold, uint8_t *use)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !use[i]) return;
    const unsigned long long k = trials[i], y = succ[i];
    const bool stands = k > 0 && y <= k && (p[i] >= threshold ? y == k : y == 0);
    use[i] = stands ? 1 : 0;
}

hipError_t sg_confirm(hipStream_t s, const float *p, const unsigned long long *succ, const unsigned long long *trials,
                      long n, float threshold, uint8_t *use)
{
    hipLaunchKernelGGL(confirm_answers, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, succ, trials, n, threshold,
                       use);
    return hipGetLastError();
}

hipError_t sg_neighbour_gate(hipStream_t s, const float *p, const float *p6, long n, float threshold, float margin,
                             uint8_t *use)
{
    hipLaunchKernelGGL(neighbour_gate, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, p6, n, threshold, margin,
                       use);
    return hipGetLastError();
}

hipError_t sg_query(hipStream_t s, const float *x, long n, const float *mu, const float *sigma,
                    const uint16_t *W1b, const float *b1, const uint16_t *W2b, const float *b2,
                    const uint16_t *W3b, const float *b3, const float *planes, int n_planes, float hull_tol,
                    float threshold, float margin, float *p_out, uint8_t *use)
{
    // the wave-tile form needs 139 KB of LDS per block; it runs where the
    // device allows it (CDNA4: 160 KB per CU), one block per CU over all tiles
    static int staged = -1, n_blocks = 0, max_lds = 0;
    if (staged < 0) {
        int dev = 0, lds = 0, cus = 0;
        staged = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            (size_t)lds >= kWaveQueryLds &&
            hipFuncSetAttribute((const void *)mlp_query_waves, hipFuncAttributeMaxDynamicSharedMemorySize, lds) ==
                hipSuccess) {
            staged = 1;
            n_blocks = cus;
            max_lds = lds;
        }
    }
    if (staged == 1 && n >= 32L * 1024) {
        const long n_tiles = (n + 31) / 32;
        const long want = (n_tiles + kQueryWaves - 1) / kQueryWaves;
        const unsigned grid = (unsigned)(want < n_blocks ? want : n_blocks);
        // the facets that fit the block's LDS are staged there (the rest are
        // read from memory)
        int lds_planes = n_planes < kLdsPlanes ? n_planes : kLdsPlanes;
        const int room = (int)(((size_t)max_lds - kWaveQueryLds) / 16);
        if (lds_planes > room) lds_planes = room;
        const size_t lds = kWaveQueryLds + (size_t)lds_planes * 16;
        hipLaunchKernelGGL(mlp_query_waves, dim3(grid), dim3(64 * kQueryWaves), lds, s, x, n, mu, sigma,
                           W1b, b1, W2b, b2, W3b, b3, planes, n_planes, lds_planes, hull_tol, threshold, margin,
                           p_out, use);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(mlp_query, dim3(blocks_for(n, 32)), dim3(256), 0, s, x, n, mu, sigma, W1b, b1, W2b, b2,
                       W3b, b3, planes, n_planes, hull_tol, threshold, margin, p_out, use);
    return hipGetLastError();
}

}  // namespace smc
