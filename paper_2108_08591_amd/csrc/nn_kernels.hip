// nn_kernels.hip -- gfx950 kernels of the convolutional encoder-decoder used
// to warm-start steady MDF-LBM solves (C ABI: include/mdfnn.h).
//
// 3x3 convolutions are implicit GEMMs on the matrix cores:
//   forward / data gradient:  M = pixels, N = output channels, K = 9 * cin,
//   weight gradient:          M = cout,   N = cin (per tap),   K = pixels,
// each a sum of v_mfma_f32_16x16x32_bf16 products (BF16 operands, FP32
// accumulation).  For that instruction lane l of a wave holds
//   A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16]   (j = 0..7)
//   C[4 (l / 16) + r][l % 16]                              (r = 0..3).
// Activations are NHWC, so one K step of 32 of the forward product (one
// tap, 32 consecutive channels) is one 16-byte chunk per pixel and weight
// row, staged through LDS as [row][32 channels]; the weight gradient, whose
// K steps are 32 pixels, stages its tiles transposed ([channel][pixel]).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mdfnn.h"

namespace mdfnn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint16_t f2bf(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8()
{
    const uint4 v = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, v);
}

// ------------------------------------------------------------------ conv fwd

// LDS-staged implicit GEMM for the forward and data-gradient products.
// Block: 4 waves, a 128-pixel x BN-channel output tile; wave (wm, wn) owns
// pixels [64 wm, +64) and channels [wn BN/2, +BN/2) as 4 x (BN/32) MFMA
// blocks of 16 x 16.  Each K step (one tap, 32 input channels) stages the
// shifted 128 x 32 input tile and the BN x 32 weight tile in LDS, every
// global value read once per block; the next step's global loads are
// issued before the current step's products (double-buffered LDS, one
// barrier per step).  Rows of the LDS tiles are 32 + 8 values long, so
// the 16 rows one MFMA operand reads start in distinct banks.
constexpr int kCvBM = 128;
constexpr int kCvLd = 40;

template <int BN>
__global__ void __launch_bounds__(256)
k_conv_fwd_lds(const uint16_t *__restrict__ x1, int c1, const uint16_t *__restrict__ x2, int c2,
               const uint16_t *__restrict__ w, const float *__restrict__ bias, int B, int H, int W, int cout,
               int relu, const uint16_t *__restrict__ mask, uint16_t *__restrict__ yb, float *__restrict__ yf)
{
    constexpr int NBW = BN / 32;                 // 16-wide channel blocks per wave
    __shared__ uint4 sA4[2][kCvBM * kCvLd / 8];
    __shared__ uint4 sB4[2][BN * kCvLd / 8];
    const int cin = c1 + c2;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i = lane & 15, g = lane >> 4, wm = wave >> 1, wn = wave & 1;
    const long long M = (long long)B * H * W;
    const long long pbase = (long long)blockIdx.x * kCvBM;
    const int co0 = blockIdx.y * BN;
    // staging roles: input rows (2 per thread: pixel t / 4 and t / 4 + 64,
    // channel chunk t % 4), weight rows (co = idx / 4, chunk idx % 4)
    const int ach = t & 3;
    int spb[2], spy[2], spx[2];
    bool spv[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const long long p = pbase + (t >> 2) + 64 * r;
        spv[r] = p < M;
        const long long pp = spv[r] ? p : 0;
        spb[r] = (int)(pp / ((long long)H * W));
        const int rem = (int)(pp % ((long long)H * W));
        spy[r] = rem / W;
        spx[r] = rem % W;
    }
    const int nk = 9 * (cin / 32);
    uint4 ra[2], rb0 = uint4{0u, 0u, 0u, 0u}, rb1 = uint4{0u, 0u, 0u, 0u};
    auto fetch = [&](int ks) __attribute__((always_inline)) {
        const int tap = ks / (cin / 32), c0 = (ks % (cin / 32)) * 32;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const uint16_t *src = (c0 < c1) ? x1 : x2;
        const int cs = (c0 < c1) ? c1 : c2;
        const int cc = (c0 < c1) ? c0 : c0 - c1;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int yy = spy[r] + dy, xx = spx[r] + dx;
            ra[r] = uint4{0u, 0u, 0u, 0u};
            if (spv[r] && yy >= 0 && yy < H && xx >= 0 && xx < W)
                ra[r] = *reinterpret_cast<const uint4 *>(src + (((long long)spb[r] * H + yy) * W + xx) * cs + cc +
                                                        8 * ach);
        }
        const uint16_t *wk = w + (long long)tap * cin + c0 + 8 * (t & 3);
        if (BN * 4 >= 256 || t < BN * 4) rb0 = *reinterpret_cast<const uint4 *>(wk + (long long)(co0 + (t >> 2)) * 9 * cin);
        if constexpr (BN * 4 > 256)
            rb1 = *reinterpret_cast<const uint4 *>(wk + (long long)(co0 + 64 + (t >> 2)) * 9 * cin);
    };
    auto stash = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < 2; ++r) sA4[buf][((t >> 2) + 64 * r) * (kCvLd / 8) + ach] = ra[r];
        if (BN * 4 >= 256 || t < BN * 4) sB4[buf][(t >> 2) * (kCvLd / 8) + (t & 3)] = rb0;
        if constexpr (BN * 4 > 256) sB4[buf][(64 + (t >> 2)) * (kCvLd / 8) + (t & 3)] = rb1;
    };
    f32x4 acc[4][NBW];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    stash(0);
    __syncthreads();
    for (int ks = 0; ks < nk; ++ks) {
        const int buf = ks & 1;
        if (ks + 1 < nk) fetch(ks + 1);
        bf16x8 fa[4], fb[NBW];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            fa[mb] = __builtin_bit_cast(bf16x8, sA4[buf][(wm * 64 + 16 * mb + i) * (kCvLd / 8) + g]);
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
            fb[nb] = __builtin_bit_cast(bf16x8, sB4[buf][(wn * (BN / 2) + 16 * nb + i) * (kCvLd / 8) + g]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mb], fb[nb], acc[mb][nb], 0, 0, 0);
        if (ks + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long p = pbase + wm * 64 + 16 * mb + 4 * g + r;
                const int co = co0 + wn * (BN / 2) + 16 * nb + i;
                if (p >= M) continue;
                float v = acc[mb][nb][r];
                if (bias) v += bias[co];
                if (relu) v = v > 0.f ? v : 0.f;
                const long long k = p * cout + co;
                if (mask && !(bf2f(mask[k]) > 0.f)) v = 0.f;
                if (yb) yb[k] = f2bf(v);
                if (yf) yf[k] = v;
            }
}

// wt[ci][tap][co] = w[co][8 - tap][ci]
__global__ void __launch_bounds__(256) k_flip(const uint16_t *__restrict__ w, int cout, int cin, uint16_t *__restrict__ wt)
{
    const long long n = (long long)cout * 9 * cin;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int ci = (int)(k / (9LL * cout));
        const int rem = (int)(k % (9LL * cout));
        const int tap = rem / cout, co = rem % cout;
        wt[k] = w[((long long)co * 9 + (8 - tap)) * cin + ci];
    }
}

// ------------------------------------------------------------------ weight grad

constexpr int kWgBlocks = 1024;    // target blocks of one weight-gradient launch

// Weight gradient with all nine taps in one block.  The K dimension (pixels)
// is walked in segments of 32 consecutive pixels of one image row; per
// segment the block stages, transposed to [channel][pixel] in LDS so that
// every MFMA operand is one 16-byte read, the output-gradient row segment
// (MT channels) once and the input window of rows y-1..y+1 (NT channels)
// in three copies shifted by dx = -1, 0, +1, and takes the products of all
// nine taps from them: each dy value is read from global memory once per
// block instead of once per tap.  Wave (wm, wn) owns channels
// [wm MT/2, +MT/2) x [wn NT/2, +NT/2) of every tap.  Pixels beyond the row
// end contribute zero (their dy is staged as zero); input pixels outside the
// image are zero.  Segments [s0, s1) of split blockIdx.z; partial sums per
// split are reduced in a fixed order by k_wgrad_reduce.
template <int MT, int NT>
__global__ void __launch_bounds__(256)
k_conv_wgrad9(const uint16_t *__restrict__ x1, int c1, const uint16_t *__restrict__ x2, int c2,
              const uint16_t *__restrict__ dyp, int B, int H, int W, int cout, int nsplit,
              float *__restrict__ partial, float *__restrict__ bpart)
{
    constexpr int MB = MT / 32, NB = NT / 32;
    constexpr int LD = 40;                              // row: 32 pixels + 8 pad
    constexpr int NDY = 32 * MT / 8;                    // 16-byte dy chunks per segment
    constexpr int NX = 3 * 34 * NT / 8;                 // 16-byte input chunks per window
    constexpr int KX = (NX + 255) / 256;
    __shared__ uint16_t ys[MT * LD];
    __shared__ uint16_t xw[9 * NT * LD];                // [dx + 1][row][ci][pixel]
    const int cin = c1 + c2;
    const int co0 = blockIdx.x * MT, ci0 = blockIdx.y * NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i = lane & 15, g = lane >> 4, wm = wave >> 1, wn = wave & 1;
    const uint16_t *src = (ci0 < c1) ? x1 : x2;
    const int cs = (ci0 < c1) ? c1 : c2;
    const int cc = (ci0 < c1) ? ci0 : ci0 - c1;
    const int S = (W + 31) / 32;                        // segments per image row
    const long long nseg = (long long)B * H * S;
    const long long per = (nseg + nsplit - 1) / nsplit;
    const long long s0 = blockIdx.z * per, s1 = (s0 + per < nseg) ? s0 + per : nseg;
    f32x4 acc[9][MB][NB];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[k][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint4 rdy, rx[KX];
    // bias gradient (blocks of the first input-channel tile): the thread that
    // stages dy chunk (pixel j, channels 8 c8 ..) sums those channels over the
    // block's segments; the 32 pixel slots are added in order at the end
    const bool bias = bpart != nullptr && blockIdx.y == 0;
    float bacc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) bacc[e] = 0.f;
    auto fetch = [&](long long sg) __attribute__((always_inline)) {
        const int xs = (int)(sg % S) * 32;
        const long long row = sg / S;                   // b * H + y
        const int y = (int)(row % H);
        rdy = uint4{0u, 0u, 0u, 0u};
        if (t < NDY) {
            const int j = t / (MT / 8), c8 = t % (MT / 8);
            if (xs + j < W) rdy = *reinterpret_cast<const uint4 *>(dyp + (row * W + xs + j) * cout + co0 + 8 * c8);
        }
#pragma unroll
        for (int r = 0; r < KX; ++r) {
            const int idx = t + 256 * r;
            rx[r] = uint4{0u, 0u, 0u, 0u};
            if (idx < NX) {
                const int wr = idx / (34 * NT / 8), rem = idx % (34 * NT / 8);
                const int c = rem / (NT / 8), c8 = rem % (NT / 8);
                const int yy = y - 1 + wr, xx = xs - 1 + c;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    rx[r] = *reinterpret_cast<const uint4 *>(src + ((row - y + yy) * W + xx) * cs + cc + 8 * c8);
            }
        }
    };
    auto stash = [&]() __attribute__((always_inline)) {
        if (t < NDY) {
            const int j = t / (MT / 8), c8 = t % (MT / 8);
            const uint16_t *u = reinterpret_cast<const uint16_t *>(&rdy);
#pragma unroll
            for (int e = 0; e < 8; ++e) ys[(8 * c8 + e) * LD + j] = u[e];
            if (bias) {
#pragma unroll
                for (int e = 0; e < 8; ++e) bacc[e] += bf2f(u[e]);
            }
        }
#pragma unroll
        for (int r = 0; r < KX; ++r) {
            const int idx = t + 256 * r;
            if (idx >= NX) continue;
            const int wr = idx / (34 * NT / 8), rem = idx % (34 * NT / 8);
            const int c = rem / (NT / 8), c8 = rem % (NT / 8);
            const uint16_t *u = reinterpret_cast<const uint16_t *>(&rx[r]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {               // copy d holds x[xs + j + d - 1]
                const int j = c + 1 - d - 1 + 0;        // pixel c of the window is xs - 1 + c
                if (j < 0 || j >= 32) continue;
#pragma unroll
                for (int e = 0; e < 8; ++e) xw[((d * 3 + wr) * NT + 8 * c8 + e) * LD + j] = u[e];
            }
        }
    };
    if (s0 < s1) fetch(s0);
    for (long long sg = s0; sg < s1; ++sg) {
        __syncthreads();                                // the previous segment's reads are done
        stash();
        __syncthreads();
        if (sg + 1 < s1) fetch(sg + 1);
        bf16x8 fa[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            fa[mb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&ys[(wm * (MT / 2) + 16 * mb + i) * LD + 8 * g]));
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int wr = tap / 3, d = tap % 3;        // dy = wr - 1, dx = d - 1
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const bf16x8 fb = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(&xw[((d * 3 + wr) * NT + wn * (NT / 2) + 16 * nb + i) * LD + 8 * g]));
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[tap][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mb], fb, acc[tap][mb][nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = co0 + wm * (MT / 2) + 16 * mb + 4 * g + r;
                    const int ci = ci0 + wn * (NT / 2) + 16 * nb + i;
                    partial[(((long long)blockIdx.z * cout + co) * 9 + tap) * cin + ci] = acc[tap][mb][nb][r];
                }
    if (bias) {
        __syncthreads();                                // xw is free: reuse it as [pixel slot][co] floats
        float *red = reinterpret_cast<float *>(xw);
        static_assert(32 * MT * sizeof(float) <= sizeof(xw), "bias slots fit the input window");
        if (t < NDY) {
            const int j = t / (MT / 8), c8 = t % (MT / 8);
#pragma unroll
            for (int e = 0; e < 8; ++e) red[j * MT + 8 * c8 + e] = bacc[e];
        }
        __syncthreads();
        if (t < MT) {
            float sum = 0.f;
            for (int j = 0; j < 32; ++j) sum += red[j * MT + t];
            bpart[(long long)blockIdx.z * cout + co0 + t] = sum;
        }
    }
}

// Sums of split partials: out[g][k] = sum of partial[sp][k] over the splits
// sp of group g = blockIdx.y ([g chunk, (g + 1) chunk)), added in split
// order.  One group (chunk >= nsplit) gives the final sums; with several, a
// second pass over the group sums adds them in group order, so the result
// is the same fixed-order sum whatever the launch.
__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float *__restrict__ partial, long long n, int nsplit, int chunk, float *__restrict__ out)
{
    const int g = blockIdx.y;
    const int sp0 = g * chunk, sp1 = (sp0 + chunk < nsplit) ? sp0 + chunk : nsplit;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        float s = 0.f;
        for (int sp = sp0; sp < sp1; ++sp) s += partial[sp * n + k];
        out[g * n + k] = s;
    }
}

// ------------------------------------------------------------------ elementwise

__global__ void __launch_bounds__(256)
k_avgpool2_fwd(const uint16_t *__restrict__ x, int B, int H, int W, int C, uint16_t *__restrict__ y)
{
    const int Ho = H / 2, Wo = W / 2;
    const long long n = (long long)B * Ho * Wo * C;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int c = (int)(k % C);
        long long q = k / C;
        const int j = (int)(q % Wo);
        q /= Wo;
        const int i = (int)(q % Ho);
        const int b = (int)(q / Ho);
        const long long base = (((long long)b * H + 2 * i) * W + 2 * j) * C + c;
        const float s = bf2f(x[base]) + bf2f(x[base + C]) + bf2f(x[base + (long long)W * C]) +
                        bf2f(x[base + (long long)W * C + C]);
        y[k] = f2bf(0.25f * s);
    }
}

__global__ void __launch_bounds__(256)
k_avgpool2_bwd(const uint16_t *__restrict__ dy, int B, int H, int W, int C, uint16_t *__restrict__ dx)
{
    const long long n = (long long)B * H * W * C;
    const int Ho = H / 2, Wo = W / 2;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int c = (int)(k % C);
        long long q = k / C;
        const int xx = (int)(q % W);
        q /= W;
        const int yy = (int)(q % H);
        const int b = (int)(q / H);
        dx[k] = f2bf(0.25f * bf2f(dy[(((long long)b * Ho + yy / 2) * Wo + xx / 2) * C + c]));
    }
}

__global__ void __launch_bounds__(256)
k_upsample2_fwd(const uint16_t *__restrict__ x, int B, int H, int W, int C, uint16_t *__restrict__ y)
{
    const int H2 = 2 * H, W2 = 2 * W;
    const long long n = (long long)B * H2 * W2 * C;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int c = (int)(k % C);
        long long q = k / C;
        const int xx = (int)(q % W2);
        q /= W2;
        const int yy = (int)(q % H2);
        const int b = (int)(q / H2);
        y[k] = x[(((long long)b * H + yy / 2) * W + xx / 2) * C + c];
    }
}

__global__ void __launch_bounds__(256)
k_upsample2_bwd(const uint16_t *__restrict__ dy, int B, int H, int W, int C, uint16_t *__restrict__ dx)
{
    const int W2 = 2 * W;
    const long long n = (long long)B * H * W * C;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int c = (int)(k % C);
        long long q = k / C;
        const int j = (int)(q % W);
        q /= W;
        const int i = (int)(q % H);
        const int b = (int)(q / H);
        const long long base = (((long long)b * 2 * H + 2 * i) * W2 + 2 * j) * C + c;
        const float s = bf2f(dy[base]) + bf2f(dy[base + C]) + bf2f(dy[base + (long long)W2 * C]) +
                        bf2f(dy[base + (long long)W2 * C + C]);
        dx[k] = f2bf(s);
    }
}

__global__ void __launch_bounds__(256)
k_add(const uint16_t *a, const uint16_t *b, const uint16_t *mask, long long n, uint16_t *out)
{
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        float v = bf2f(a[k]);
        if (b) v += bf2f(b[k]);
        if (mask && !(bf2f(mask[k]) > 0.f)) v = 0.f;
        out[k] = f2bf(v);
    }
}

// ------------------------------------------------------------------ 1x1 head

__global__ void __launch_bounds__(256)
k_head_fwd(const uint16_t *__restrict__ x, int P, int cin, const float *__restrict__ w,
           const float *__restrict__ bias, int cout, float *__restrict__ y)
{
    __shared__ float sw[32 * 32];
    __shared__ float sb[32];
    for (int k = threadIdx.x; k < cout * cin; k += 256) sw[k] = w[k];
    if (threadIdx.x < cout) sb[threadIdx.x] = bias ? bias[threadIdx.x] : 0.f;
    __syncthreads();
    const long long p = blockIdx.x * 256LL + threadIdx.x;
    if (p >= P) return;
    float xv[32];
    for (int c = 0; c < cin; ++c) xv[c] = bf2f(x[p * cin + c]);
    for (int o = 0; o < cout; ++o) {
        float s = sb[o];
        for (int c = 0; c < cin; ++c) s += sw[o * cin + c] * xv[c];
        y[p * cout + o] = s;
    }
}

__global__ void __launch_bounds__(256)
k_head_bwd_x(const float *__restrict__ dy, int P, int cin, const float *__restrict__ w, int cout,
             const uint16_t *__restrict__ mask, uint16_t *__restrict__ dx)
{
    __shared__ float sw[32 * 32];
    for (int k = threadIdx.x; k < cout * cin; k += 256) sw[k] = w[k];
    __syncthreads();
    const long long p = blockIdx.x * 256LL + threadIdx.x;
    if (p >= P) return;
    for (int c = 0; c < cin; ++c) {
        float s = 0.f;
        for (int o = 0; o < cout; ++o) s += dy[p * cout + o] * sw[o * cin + c];
        if (mask && !(bf2f(mask[p * cin + c]) > 0.f)) s = 0.f;
        dx[p * cin + c] = f2bf(s);
    }
}

// one thread per (o, c) pair (and per o for the bias), a pixel range per block
__global__ void __launch_bounds__(256)
k_head_bwd_w(const uint16_t *__restrict__ x, const float *__restrict__ dy, int P, int cin, int cout,
             int rows_per_block, float *__restrict__ partial)
{
    const int t = threadIdx.x;
    const int nw = cout * cin;
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const long long r1 = (r0 + rows_per_block < P) ? r0 + rows_per_block : P;
    if (t < nw) {
        const int o = t / cin, c = t % cin;
        float s = 0.f;
        for (long long p = r0; p < r1; ++p) s += dy[p * cout + o] * bf2f(x[p * cin + c]);
        partial[(long long)blockIdx.x * (nw + cout) + t] = s;
    } else if (t < nw + cout) {
        const int o = t - nw;
        float s = 0.f;
        for (long long p = r0; p < r1; ++p) s += dy[p * cout + o];
        partial[(long long)blockIdx.x * (nw + cout) + t] = s;
    }
}

__global__ void __launch_bounds__(256)
k_head_bwd_reduce(const float *__restrict__ partial, int nblk, int cin, int cout, float *__restrict__ dw,
                  float *__restrict__ db)
{
    const int t = threadIdx.x;
    const int nw = cout * cin;
    if (t >= nw + cout) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += partial[(long long)b * (nw + cout) + t];
    if (t < nw) dw[t] = s;
    else if (db) db[t - nw] = s;
}

// ------------------------------------------------------------------ loss, optimiser

// pass 1: per-block partial sums of wt (d^2 summed over channels) and wt
__global__ void __launch_bounds__(256)
k_mse_partial(const float *__restrict__ y, const float *__restrict__ tg, const float *__restrict__ wt, int P,
              int C, float *__restrict__ partial)
{
    __shared__ float s1[256], s2[256];
    const long long p = blockIdx.x * 256LL + threadIdx.x;
    float a = 0.f, b = 0.f;
    if (p < P) {
        const float ww = wt[p];
        for (int c = 0; c < C; ++c) {
            const float d = y[p * C + c] - tg[p * C + c];
            a += ww * d * d;
        }
        b = ww;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s1[0];
        partial[2 * blockIdx.x + 1] = s2[0];
    }
}

// pass 2 (one block): totals; loss = S / (Wsum C); totals kept for pass 3
__global__ void __launch_bounds__(256)
k_mse_total(const float *__restrict__ partial, int nblk, int C, float *__restrict__ totals, float *__restrict__ loss)
{
    __shared__ float s1[256], s2[256];
    float a = 0.f, b = 0.f;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = s1[0];
        totals[1] = s2[0];
        if (loss) *loss = s2[0] > 0.f ? s1[0] / (s2[0] * C) : 0.f;
    }
}

// pass 3: dy = 2 wt (y - t) / (Wsum C)
__global__ void __launch_bounds__(256)
k_mse_grad(const float *__restrict__ y, const float *__restrict__ tg, const float *__restrict__ wt, int P, int C,
           const float *__restrict__ totals, float *__restrict__ dy)
{
    const long long p = blockIdx.x * 256LL + threadIdx.x;
    if (p >= P) return;
    const float den = totals[1] * C;
    const float sc = den > 0.f ? 2.f * wt[p] / den : 0.f;
    for (int c = 0; c < C; ++c) dy[p * C + c] = sc * (y[p * C + c] - tg[p * C + c]);
}

__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v, long long n,
       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *__restrict__ pb)
{
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.f - b1) * gk;
        const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        const float mh = mk / c1, vh = vk / c2;
        const float pk = p[k] - lr * mh / (sqrtf(vh) + eps);
        p[k] = pk;
        if (pb) pb[k] = f2bf(pk);
    }
}

__global__ void __launch_bounds__(256) k_to_bf16(const float *__restrict__ x, long long n, uint16_t *__restrict__ y)
{
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) y[k] = f2bf(x[k]);
}

__global__ void __launch_bounds__(256) k_to_f32(const uint16_t *__restrict__ x, long long n, float *__restrict__ y)
{
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) y[k] = bf2f(x[k]);
}

int grid1(long long n)
{
    long long g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

int status(hipError_t e) { return e == hipSuccess ? MDFNN_OK : MDFNN_EDEVICE; }

}  // namespace
}  // namespace mdfnn

using namespace mdfnn;

extern "C" {

int mdfnn_conv3x3_fwd(const uint16_t *x1, int c1, const uint16_t *x2, int c2, const uint16_t *w,
                      const float *bias, int B, int H, int W, int cout, int relu, const uint16_t *mask,
                      uint16_t *y_bf16, float *y_f32, void *stream)
{
    if (!x1 || !w || (!y_bf16 && !y_f32) || B < 1 || H < 1 || W < 1) return MDFNN_EINVAL;
    if (c1 < 32 || c1 % 32 || c2 < 0 || c2 % 32 || (c2 > 0 && !x2) || cout < 32 || cout % 32) return MDFNN_EINVAL;
    const long long M = (long long)B * H * W;
    if (M > (1LL << 31)) return MDFNN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned gx = (unsigned)((M + kCvBM - 1) / kCvBM);
    if (cout % 128 == 0)
        hipLaunchKernelGGL(k_conv_fwd_lds<128>, dim3(gx, cout / 128), dim3(256), 0, st, x1, c1, x2, c2, w, bias, B, H,
                           W, cout, relu, mask, y_bf16, y_f32);
    else if (cout % 64 == 0)
        hipLaunchKernelGGL(k_conv_fwd_lds<64>, dim3(gx, cout / 64), dim3(256), 0, st, x1, c1, x2, c2, w, bias, B, H, W,
                           cout, relu, mask, y_bf16, y_f32);
    else
        hipLaunchKernelGGL(k_conv_fwd_lds<32>, dim3(gx, cout / 32), dim3(256), 0, st, x1, c1, x2, c2, w, bias, B, H, W,
                           cout, relu, mask, y_bf16, y_f32);
    return status(hipGetLastError());
}

int mdfnn_conv3x3_flip(const uint16_t *w, int cout, int cin, uint16_t *wt, void *stream)
{
    if (!w || !wt || cout < 1 || cin < 1) return MDFNN_EINVAL;
    const long long n = (long long)cout * 9 * cin;
    hipLaunchKernelGGL(k_flip, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), w, cout, cin, wt);
    return status(hipGetLastError());
}

// Channel tiles of the weight gradient: MT output x NT input channels; a
// tile of input channels must not straddle x1 and x2.
static int wgrad_mt(int cout) { return (cout % 64 == 0) ? 64 : 32; }
static int wgrad_nt(int c1, int c2) { return (c1 % 64 == 0 && c2 % 64 == 0) ? 64 : 32; }

// Splits of the pixel segments (32 pixels of one image row each): about 1024
// blocks over the channel tiles, at least 8 segments per split.
static int wgrad_splits(int B, int H, int W, int ntiles)
{
    const long long nseg = (long long)B * H * ((W + 31) / 32);
    long long s = (kWgBlocks + ntiles - 1) / ntiles;
    if (s > nseg / 8) s = nseg / 8;
    if (s < 1) s = 1;
    return (int)s;
}

// Splits per group of the first reduction pass.
constexpr int kWgChunk = 32;

// Fixed-order sum over ns split partials of n values each (two passes when
// ns > kWgChunk, through mid: ceil(ns / kWgChunk) * n floats).
static hipError_t reduce_splits(const float *partial, long long n, int ns, float *mid, float *out, hipStream_t st)
{
    if (ns <= kWgChunk) {
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid1(n), 1), dim3(256), 0, st, partial, n, ns, ns, out);
        return hipGetLastError();
    }
    const int G = (ns + kWgChunk - 1) / kWgChunk;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid1(n), G), dim3(256), 0, st, partial, n, ns, kWgChunk, mid);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid1(n), 1), dim3(256), 0, st, mid, n, G, G, out);
    return hipGetLastError();
}

size_t mdfnn_wgrad_scratch_bytes(int B, int H, int W, int cin, int cout)
{
    if (B < 1 || H < 1 || W < 1 || cin < 32 || cout < 32) return 0;
    // the smallest tiles give the most splits
    const int ns = wgrad_splits(B, H, W, (cout / 64 > 0 ? cout / 64 : 1) * (cin / 64 > 0 ? cin / 64 : 1));
    const size_t G = (size_t)(ns + kWgChunk - 1) / kWgChunk;
    const size_t n = (size_t)cout * 9 * cin;
    // weight and bias partials, then the group sums of both
    return ((size_t)ns * (n + cout) + G * (n + cout)) * sizeof(float) + 256;
}

int mdfnn_conv3x3_wgrad(const uint16_t *x1, int c1, const uint16_t *x2, int c2, const uint16_t *dy, int B, int H,
                        int W, int cout, float *dw, float *db, void *scratch, void *stream)
{
    if (!x1 || !dy || !dw || !scratch || B < 1 || H < 1 || W < 1) return MDFNN_EINVAL;
    const int cin = c1 + c2;
    if (c1 < 32 || c1 % 32 || c2 < 0 || c2 % 32 || (c2 > 0 && !x2) || cout < 32 || cout % 32) return MDFNN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mt = wgrad_mt(cout), nt = wgrad_nt(c1, c2);
    const int ns = wgrad_splits(B, H, W, (cout / mt) * (cin / nt));
    float *wpart = static_cast<float *>(scratch);
    float *bpart = db ? wpart + (size_t)ns * cout * 9 * cin : nullptr;
    const dim3 grid(cout / mt, cin / nt, ns);
    if (mt == 64 && nt == 64)
        hipLaunchKernelGGL((k_conv_wgrad9<64, 64>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart,
                           bpart);
    else if (mt == 64)
        hipLaunchKernelGGL((k_conv_wgrad9<64, 32>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart,
                           bpart);
    else if (nt == 64)
        hipLaunchKernelGGL((k_conv_wgrad9<32, 64>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart,
                           bpart);
    else
        hipLaunchKernelGGL((k_conv_wgrad9<32, 32>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart,
                           bpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return MDFNN_EDEVICE;
    const long long n = (long long)cout * 9 * cin;
    float *mid = wpart + (size_t)ns * (n + cout);
    e = reduce_splits(wpart, n, ns, mid, dw, st);
    if (e != hipSuccess) return MDFNN_EDEVICE;
    if (db) e = reduce_splits(bpart, cout, ns, mid + (size_t)((ns + kWgChunk - 1) / kWgChunk) * n, db, st);
    return status(e);
}

int mdfnn_avgpool2_fwd(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, void *stream)
{
    if (!x || !y || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1) return MDFNN_EINVAL;
    const long long n = (long long)B * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_avgpool2_fwd, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, B, H, W, C, y);
    return status(hipGetLastError());
}

int mdfnn_avgpool2_bwd(const uint16_t *dy, int B, int H, int W, int C, uint16_t *dx, void *stream)
{
    if (!dy || !dx || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1) return MDFNN_EINVAL;
    const long long n = (long long)B * H * W * C;
    hipLaunchKernelGGL(k_avgpool2_bwd, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), dy, B, H, W, C, dx);
    return status(hipGetLastError());
}

int mdfnn_upsample2_fwd(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, void *stream)
{
    if (!x || !y || B < 1 || H < 1 || W < 1 || C < 1) return MDFNN_EINVAL;
    const long long n = (long long)B * 4 * H * W * C;
    hipLaunchKernelGGL(k_upsample2_fwd, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, B, H, W, C, y);
    return status(hipGetLastError());
}

int mdfnn_upsample2_bwd(const uint16_t *dy, int B, int H, int W, int C, uint16_t *dx, void *stream)
{
    if (!dy || !dx || B < 1 || H < 1 || W < 1 || C < 1) return MDFNN_EINVAL;
    const long long n = (long long)B * H * W * C;
    hipLaunchKernelGGL(k_upsample2_bwd, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), dy, B, H, W, C, dx);
    return status(hipGetLastError());
}

int mdfnn_add(const uint16_t *a, const uint16_t *b, const uint16_t *mask, long long n, uint16_t *out, void *stream)
{
    if (!a || !out || n < 0) return MDFNN_EINVAL;
    hipLaunchKernelGGL(k_add, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), a, b, mask, n, out);
    return status(hipGetLastError());
}

int mdfnn_head_fwd(const uint16_t *x, int P, int cin, const float *w, const float *bias, int cout, float *y,
                   void *stream)
{
    if (!x || !w || !y || P < 1 || cin < 1 || cin > 32 || cout < 1 || cout > 32) return MDFNN_EINVAL;
    hipLaunchKernelGGL(k_head_fwd, dim3((P + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), x, P, cin, w,
                       bias, cout, y);
    return status(hipGetLastError());
}

size_t mdfnn_head_scratch_bytes(int P, int cin, int cout)
{
    const int rows = 512;
    const size_t nblk = (size_t)((P + rows - 1) / rows);
    return nblk * (size_t)(cin * cout + cout) * sizeof(float) + 256;
}

int mdfnn_head_bwd(const uint16_t *x, const float *dy, int P, int cin, const float *w, int cout, const uint16_t *mask,
                   uint16_t *dx, float *dw, float *db, void *scratch, void *stream)
{
    if (!x || !dy || !w || !dw || !scratch || P < 1 || cin < 1 || cin > 32 || cout < 1 || cout > 32 ||
        cin * cout + cout > 256)
        return MDFNN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dx)
        hipLaunchKernelGGL(k_head_bwd_x, dim3((P + 255) / 256), dim3(256), 0, st, dy, P, cin, w, cout, mask, dx);
    const int rows = 512;
    const int nblk = (P + rows - 1) / rows;
    float *part = static_cast<float *>(scratch);
    hipLaunchKernelGGL(k_head_bwd_w, dim3(nblk), dim3(256), 0, st, x, dy, P, cin, cout, rows, part);
    hipLaunchKernelGGL(k_head_bwd_reduce, dim3(1), dim3(256), 0, st, part, nblk, cin, cout, dw, db);
    return status(hipGetLastError());
}

size_t mdfnn_loss_scratch_bytes(int P) { return (size_t)(2 * ((P + 255) / 256) + 2) * sizeof(float) + 256; }

int mdfnn_mse(const float *y, const float *t, const float *wt, int P, int C, float *dy, float *loss, void *scratch,
              void *stream)
{
    if (!y || !t || !wt || !dy || !scratch || P < 1 || C < 1) return MDFNN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblk = (P + 255) / 256;
    float *part = static_cast<float *>(scratch);
    float *totals = part + 2 * nblk;
    hipLaunchKernelGGL(k_mse_partial, dim3(nblk), dim3(256), 0, st, y, t, wt, P, C, part);
    hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(256), 0, st, part, nblk, C, totals, loss);
    hipLaunchKernelGGL(k_mse_grad, dim3(nblk), dim3(256), 0, st, y, t, wt, P, C, totals, dy);
    return status(hipGetLastError());
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free loss

namespace mdfnn {
namespace {

// Device scratch of mdfnn_mse_noalloc: the per-block partial sums and the two
// totals of the loss, for at most kMseStaticMaxP pixels.  Each GPU holds its
// own copy for the life of the process.  In host code `scratch` names a
// host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
constexpr int kMseStaticMaxP = MDFNN_MSE_NOALLOC_MAX_P;
constexpr int kMseStaticFloats = 2 * ((kMseStaticMaxP + 255) / 256) + 2;
__device__ __align__(256) float scratch[kMseStaticFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
float *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's `scratch`, looked up once per device with
// that device current.
hipError_t mse_scratch(float **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace mdfnn

extern "C" {

int mdfnn_mse_noalloc(const float *y, const float *t, const float *wt, int P, int C, float *dy, float *loss,
                      void *stream)
{
    if (!y || !t || !wt || !dy || P < 1 || C < 1) return MDFNN_EINVAL;
    if (P > kMseStaticMaxP) return MDFNN_ETOOBIG;
    float *part = nullptr;
    hipError_t e = mse_scratch(&part);
    if (e != hipSuccess) return MDFNN_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblk = (P + 255) / 256;
    float *totals = part + 2 * nblk;
    // every partial and both totals are written before they are read: nothing
    // left by an earlier call is used
    hipLaunchKernelGGL(k_mse_partial, dim3(nblk), dim3(256), 0, st, y, t, wt, P, C, part);
    hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(256), 0, st, part, nblk, C, totals, loss);
    hipLaunchKernelGGL(k_mse_grad, dim3(nblk), dim3(256), 0, st, y, t, wt, P, C, totals, dy);
    return status(hipGetLastError());
}

int mdfnn_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps, int t,
               uint16_t *p_bf16, void *stream)
{
    if (!p || !g || !m || !v || n < 0 || t < 1) return MDFNN_EINVAL;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g, m, v, n, lr, b1, b2,
                       eps, c1, c2, p_bf16);
    return status(hipGetLastError());
}

int mdfnn_to_bf16(const float *x, long long n, uint16_t *y, void *stream)
{
    if (!x || !y || n < 0) return MDFNN_EINVAL;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, n, y);
    return status(hipGetLastError());
}

int mdfnn_to_f32(const uint16_t *x, long long n, float *y, void *stream)
{
    if (!x || !y || n < 0) return MDFNN_EINVAL;
    hipLaunchKernelGGL(k_to_f32, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, n, y);
    return status(hipGetLastError());
}

}  // extern "C"
