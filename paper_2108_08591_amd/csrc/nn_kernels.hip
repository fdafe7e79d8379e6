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
// Activations are NHWC, so one K step of 32 (one tap, 32 consecutive
// channels) is a single 16-byte load per lane for both operands of the
// forward product; the weight gradient stages pixel tiles through LDS.
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

// Block: 4 waves, 128 pixels x (16 NB) output channels; wave w owns pixels
// [32 w, 32 w + 32) of the block as two 16-row MFMA blocks.
template <int NB>
__global__ void __launch_bounds__(256)
k_conv_fwd(const uint16_t *__restrict__ x1, int c1, const uint16_t *__restrict__ x2, int c2,
           const uint16_t *__restrict__ w, const float *__restrict__ bias, int B, int H, int W, int cout,
           int relu, const uint16_t *__restrict__ mask, uint16_t *__restrict__ yb, float *__restrict__ yf)
{
    const int cin = c1 + c2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const long long M = (long long)B * H * W;
    const long long p0 = (long long)blockIdx.x * 128 + wave * 32;
    const int co0 = blockIdx.y * (16 * NB);
    int pbb[2], py[2], px[2];
    bool pv[2];
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
        const long long p = p0 + 16 * pb + i;
        pv[pb] = p < M;
        const long long pp = pv[pb] ? p : 0;
        pbb[pb] = (int)(pp / ((long long)H * W));
        const int r = (int)(pp % ((long long)H * W));
        py[pb] = r / W;
        px[pb] = r % W;
    }
    f32x4 acc[2][NB];
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[pb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        long long off[2];
        bool in[2];
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
            const int yy = py[pb] + dy, xx = px[pb] + dx;
            in[pb] = pv[pb] && yy >= 0 && yy < H && xx >= 0 && xx < W;
            off[pb] = in[pb] ? (((long long)pbb[pb] * H + yy) * W + xx) : 0;
        }
        for (int c0 = 0; c0 < cin; c0 += 32) {
            const uint16_t *src = (c0 < c1) ? x1 : x2;
            const int cs = (c0 < c1) ? c1 : c2;
            const int cc = (c0 < c1) ? c0 : c0 - c1;
            bf16x8 a[2];
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) a[pb] = in[pb] ? load8(src + off[pb] * cs + cc + 8 * g) : zero8();
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const int co = co0 + 16 * cb + i;
                const bf16x8 b = load8(w + ((long long)co * 9 + tap) * cin + c0 + 8 * g);
#pragma unroll
                for (int pb = 0; pb < 2; ++pb)
                    acc[pb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pb], b, acc[pb][cb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long p = p0 + 16 * pb + 4 * g + r;
                const int co = co0 + 16 * cb + i;
                if (p >= M) continue;
                float v = acc[pb][cb][r];
                if (bias) v += bias[co];
                if (relu) v = v > 0.f ? v : 0.f;
                const long long k = p * cout + co;
                if (mask && !(bf2f(mask[k]) > 0.f)) v = 0.f;
                if (yb) yb[k] = f2bf(v);
                if (yf) yf[k] = v;
            }
}

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
    constexpr int BCH = BN * 4 / 256;            // 16-byte weight chunks per thread (BN >= 64)
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
    uint4 ra[2], rb[BCH > 0 ? BCH : 1];
    auto fetch = [&](int ks) {
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
        if constexpr (BCH > 0) {
#pragma unroll
            for (int r = 0; r < BCH; ++r) {
                const int idx = t + 256 * r;
                const int co = co0 + (idx >> 2);
                rb[r] = *reinterpret_cast<const uint4 *>(w + ((long long)co * 9 + tap) * cin + c0 + 8 * (idx & 3));
            }
        } else {
            if (t < BN * 4) {
                const int co = co0 + (t >> 2);
                rb[0] = *reinterpret_cast<const uint4 *>(w + ((long long)co * 9 + tap) * cin + c0 + 8 * (t & 3));
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 2; ++r) sA4[buf][((t >> 2) + 64 * r) * (kCvLd / 8) + ach] = ra[r];
        if constexpr (BCH > 0) {
#pragma unroll
            for (int r = 0; r < BCH; ++r) {
                const int idx = t + 256 * r;
                sB4[buf][(idx >> 2) * (kCvLd / 8) + (idx & 3)] = rb[r];
            }
        } else {
            if (t < BN * 4) sB4[buf][(t >> 2) * (kCvLd / 8) + (t & 3)] = rb[0];
        }
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

// Block: 4 waves, an MT (cout) x NT (cin) tile of one tap over a contiguous
// range of pixels; partial sums per pixel range go to scratch and are summed
// in a fixed order by k_wgrad_reduce.  Wave (wm, wn) owns rows
// [wm MT/2, +MT/2) and columns [wn NT/2, +NT/2), as (MT/32) x (NT/32) MFMA
// blocks of 16 x 16.  MT, NT in {32, 64}.
constexpr int kWgSplitMax = 64;

template <int MT, int NT>
__global__ void __launch_bounds__(256)
k_conv_wgrad(const uint16_t *__restrict__ x1, int c1, const uint16_t *__restrict__ x2, int c2,
             const uint16_t *__restrict__ dyp, int B, int H, int W, int cout, int nsplit,
             float *__restrict__ partial)
{
    constexpr int MB = MT / 32, NB = NT / 32;
    __shared__ uint16_t sA[32][MT + 8];     // dy tile  [pixel][co]
    __shared__ uint16_t sB[32][NT + 8];     // x tile   [pixel][ci]
    const int cin = c1 + c2;
    const int nci = cin / NT;
    const int co0 = blockIdx.x * MT;
    const int tap = blockIdx.y / nci, ci0 = (blockIdx.y % nci) * NT;
    const int split = blockIdx.z;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const long long M = (long long)B * H * W;
    const long long per = (M + nsplit - 1) / nsplit;
    const long long k0 = split * per, k1 = (k0 + per < M) ? k0 + per : M;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i = lane & 15, g = lane >> 4, wm = wave >> 1, wn = wave & 1;
    const uint16_t *src = (ci0 < c1) ? x1 : x2;
    const int cs = (ci0 < c1) ? c1 : c2;
    const int cc = (ci0 < c1) ? ci0 : ci0 - c1;
    f32x4 acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (long long kb = k0; kb < k1; kb += 32) {
        // dy tile: 32 pixels x MT channels, 8 channels per load
        for (int idx = t; idx < 32 * (MT / 8); idx += 256) {
            const int lp = idx / (MT / 8), lc = (idx % (MT / 8)) * 8;
            const long long p = kb + lp;
            uint4 va = {0u, 0u, 0u, 0u};
            if (p < k1) va = *reinterpret_cast<const uint4 *>(dyp + p * cout + co0 + lc);
            const uint16_t *ua = reinterpret_cast<const uint16_t *>(&va);
#pragma unroll
            for (int j = 0; j < 8; ++j) sA[lp][lc + j] = ua[j];
        }
        // shifted input tile: 32 pixels x NT channels
        for (int idx = t; idx < 32 * (NT / 8); idx += 256) {
            const int lp = idx / (NT / 8), lc = (idx % (NT / 8)) * 8;
            const long long p = kb + lp;
            uint4 vb = {0u, 0u, 0u, 0u};
            if (p < k1) {
                const int b = (int)(p / ((long long)H * W));
                const int r = (int)(p % ((long long)H * W));
                const int yy = r / W + dy, xx = r % W + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    vb = *reinterpret_cast<const uint4 *>(src + (((long long)b * H + yy) * W + xx) * cs + cc + lc);
            }
            const uint16_t *ub = reinterpret_cast<const uint16_t *>(&vb);
#pragma unroll
            for (int j = 0; j < 8; ++j) sB[lp][lc + j] = ub[j];
        }
        __syncthreads();
        bf16x8 fa[MB], fb[NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            uint16_t tmp[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) tmp[j] = sA[8 * g + j][wm * (MT / 2) + 16 * mb + i];
            fa[mb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(tmp));
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            uint16_t tmp[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) tmp[j] = sB[8 * g + j][wn * (NT / 2) + 16 * nb + i];
            fb[nb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(tmp));
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mb], fb[nb], acc[mb][nb], 0, 0, 0);
        __syncthreads();
    }
    // partial[split][co][tap][ci]
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + wm * (MT / 2) + 16 * mb + 4 * g + r;
                const int ci = ci0 + wn * (NT / 2) + 16 * nb + i;
                partial[(((long long)split * cout + co) * 9 + tap) * cin + ci] = acc[mb][nb][r];
            }
}

__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float *__restrict__ partial, long long n, int nsplit, float *__restrict__ dw)
{
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        float s = 0.f;
        for (int sp = 0; sp < nsplit; ++sp) s += partial[sp * n + k];
        dw[k] = s;
    }
}

// Column sums of a bf16 [P][C] matrix: partial[block][c], then fixed-order sum.
__global__ void __launch_bounds__(256)
k_colsum_partial(const uint16_t *__restrict__ x, long long P, int C, int rows_per_block, float *__restrict__ partial)
{
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const long long r1 = (r0 + rows_per_block < P) ? r0 + rows_per_block : P;
    for (int c = threadIdx.x; c < C; c += 256) {
        float s = 0.f;
        for (long long r = r0; r < r1; ++r) s += bf2f(x[r * C + c]);
        partial[(long long)blockIdx.x * C + c] = s;
    }
}

__global__ void __launch_bounds__(256)
k_colsum_reduce(const float *__restrict__ partial, int nblk, int C, float *__restrict__ out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += partial[(long long)b * C + c];
    out[c] = s;
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

static int wgrad_splits(long long M)
{
    long long s = (M + 4095) / 4096;
    if (s > kWgSplitMax) s = kWgSplitMax;
    if (s < 1) s = 1;
    return (int)s;
}

size_t mdfnn_wgrad_scratch_bytes(int B, int H, int W, int cin, int cout)
{
    const long long M = (long long)B * H * W;
    const int ns = wgrad_splits(M);
    const size_t wpart = (size_t)ns * cout * 9 * cin * sizeof(float);
    const int rows = 1024;
    const size_t nblk = (size_t)((M + rows - 1) / rows);
    const size_t bpart = nblk * cout * sizeof(float);
    return wpart + bpart + 256;
}

int mdfnn_conv3x3_wgrad(const uint16_t *x1, int c1, const uint16_t *x2, int c2, const uint16_t *dy, int B, int H,
                        int W, int cout, float *dw, float *db, void *scratch, void *stream)
{
    if (!x1 || !dy || !dw || !scratch || B < 1 || H < 1 || W < 1) return MDFNN_EINVAL;
    const int cin = c1 + c2;
    if (c1 < 32 || c1 % 32 || c2 < 0 || c2 % 32 || (c2 > 0 && !x2) || cout < 32 || cout % 32) return MDFNN_EINVAL;
    const long long M = (long long)B * H * W;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int ns = wgrad_splits(M);
    float *wpart = static_cast<float *>(scratch);
    // a cin tile must not straddle x1 and x2: 64-wide tiles need c1 % 64 == 0
    const int mt = (cout % 64 == 0) ? 64 : 32;
    const int nt = (c1 % 64 == 0 && c2 % 64 == 0) ? 64 : 32;
    const dim3 grid(cout / mt, 9 * (cin / nt), ns);
    if (mt == 64 && nt == 64)
        hipLaunchKernelGGL((k_conv_wgrad<64, 64>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart);
    else if (mt == 64)
        hipLaunchKernelGGL((k_conv_wgrad<64, 32>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart);
    else if (nt == 64)
        hipLaunchKernelGGL((k_conv_wgrad<32, 64>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart);
    else
        hipLaunchKernelGGL((k_conv_wgrad<32, 32>), grid, dim3(256), 0, st, x1, c1, x2, c2, dy, B, H, W, cout, ns, wpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return MDFNN_EDEVICE;
    const long long n = (long long)cout * 9 * cin;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid1(n)), dim3(256), 0, st, wpart, n, ns, dw);
    e = hipGetLastError();
    if (e != hipSuccess) return MDFNN_EDEVICE;
    if (db) {
        const int rows = 1024;
        const int nblk = (int)((M + rows - 1) / rows);
        float *bpart = wpart + (size_t)ns * cout * 9 * cin;
        hipLaunchKernelGGL(k_colsum_partial, dim3(nblk), dim3(256), 0, st, dy, M, cout, rows, bpart);
        hipLaunchKernelGGL(k_colsum_reduce, dim3((cout + 255) / 256), dim3(256), 0, st, bpart, nblk, cout, db);
        e = hipGetLastError();
    }
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
