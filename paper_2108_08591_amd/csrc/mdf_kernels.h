#pragma once
// mdf_kernels.h -- gfx950 kernels of the MDF-LBM hot path (templates).
//
// Included by one translation unit per lattice (lat_*.hip), which
// instantiates that lattice's kernels for every storage, and by
// mdf_launch.hip for the lattice-independent launch helpers.
//
// Method (Chai, Shi & Zhan, arXiv 2108.08591): d+1 distribution sets a = 0..d,
// one per convection-diffusion equation of eq. 2-2 (ubar_0 = rho0, ubar_a = u_a),
// advanced by the diffusive-scaling evolution of Remark I (eq. 3-21)
//     f_{i,a}(x + c_i, t + 1) = f_{i,a} - sum_k L_{ik} (f_{k,a} - f^eq_{k,a}) + w_i Fbar_a.
//
// Data layout in HBM (structure of arrays): one plane per (set a, direction i),
//     pop[(a*Q + i) * dstride + (z*ny + y) * pitch + x],
// x fastest, rows padded so that a row is a whole number of 128-byte lines,
// planes dstride elements apart (nz*ny*pitch and a gap of 2304 bytes).
// Two such buffers ping-pong: buffer `src` holds the post-collision state
// f*(., t) of every node, a step pulls f_{i,a}(x, t+1) = f*_{i,a}(x - c_i, t)
// (so every lane's loads of one plane are consecutive addresses), collides it
// at the node and writes f*(x, t+1) to `dst` at the same node.  One thread
// owns one node; the kernel reads and writes each population exactly once,
// so it is bound by HBM bandwidth (2 Q (d+1) s bytes per node and step).
//
// Collision: the paper's matrix L = M^{-1} S_d M (eq. 4-1..4-3) is applied in
// its exact projection form.  M has mutually orthogonal rows; S_d gives s0 to
// the conserved row e, s1 to the d velocity rows (odd under c -> -c) and s2
// to every remaining row (even), so
//     L n = s1 P_odd n + s2 P_even n + (s0 - s2) (e.n / Q) e,
// with (P_odd n)_i = (n_i - n_ibar)/2, (P_even n)_i = (n_i + n_ibar)/2 for
// i != 0, (P_odd n)_0 = 0, (P_even n)_0 = n_0.  For n = f - f^eq the last
// term vanishes (e.n = 0, eq. 3-8); see collide_fused().
//
// Walls: a link whose upstream node lies behind a wall face or in a solid
// node takes the halfway wall rule (Section 4 names an anti-bounce-back rule
// without printing it; read as)
//     a >= 1: f_{i,a}(x, t+1) = -f*_{ibar,a}(x, t) + 2 w_i U_{w,a}
//     a = 0 : f_{i,0}(x, t+1) =  f*_{ibar,0}(x, t).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mdf_internal.h"

namespace mdf {
namespace {

// ----------------------------------------------------------------- lattices

// D2Q5 (eq. d2q5) with w_0 = 1/3 as used in Section 4.  NS is the number of
// stored distribution sets and A0 the set index a of the first stored one:
// all d + 1 sets (a = 0..d), or, in the *V variants, only the d velocity
// sets a = 1..d (Remark IV: the set a = 0 only advects rho0 and no other
// quantity reads it).  R is the index of the first moving population (1
// after the rest population, 0 on lattices without one) and K the index of
// the population that closes the zeroth-moment identity of the collision
// (the rest population, else the last moving one).  w[i] is the weight of
// direction i and wc[i] its class (0 rest, 1 axis, 2 diagonal: the index of
// the case's rest-value table); DIAG marks lattices with diagonal links.
struct LatD2Q5 {
    static constexpr int D = 2, Q = 5, NS = 3, A0 = 0, R = 1, K = 0;
    static constexpr bool DIAG = false;
    static constexpr double w[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
    static constexpr int wc[5] = {0, 1, 1, 1, 1};
    static constexpr int cx[5] = {0, 1, 0, -1, 0};
    static constexpr int cy[5] = {0, 0, 1, 0, -1};
    static constexpr int cz[5] = {0, 0, 0, 0, 0};
    static constexpr int opp[5] = {0, 3, 4, 1, 2};
    static constexpr double w0 = 1.0 / 3.0, w1 = 1.0 / 6.0;
    static constexpr double cs2 = 1.0 / 3.0, inv_cs2 = 3.0;
};

// D3Q7 (eq. d3q7).
struct LatD3Q7 {
    static constexpr int D = 3, Q = 7, NS = 4, A0 = 0, R = 1, K = 0;
    static constexpr bool DIAG = false;
    static constexpr double w[7] = {1.0 / 4.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0};
    static constexpr int wc[7] = {0, 1, 1, 1, 1, 1, 1};
    static constexpr int cx[7] = {0, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[7] = {0, 0, 0, 1, -1, 0, 0};
    static constexpr int cz[7] = {0, 0, 0, 0, 0, 1, -1};
    static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
    static constexpr double w0 = 1.0 / 4.0, w1 = 1.0 / 8.0;
    static constexpr double cs2 = 1.0 / 4.0, inv_cs2 = 4.0;
};

// D2Q4 (eq. d2q4) and D3Q6 (eq. d3q6): no rest population; w0 only
// stands for a moving weight in expressions shared with the other lattices.
struct LatD2Q4 {
    static constexpr int D = 2, Q = 4, NS = 3, A0 = 0, R = 0, K = 3;
    static constexpr bool DIAG = false;
    static constexpr double w[4] = {1.0 / 4.0, 1.0 / 4.0, 1.0 / 4.0, 1.0 / 4.0};
    static constexpr int wc[4] = {1, 1, 1, 1};
    static constexpr int cx[4] = {1, 0, -1, 0};
    static constexpr int cy[4] = {0, 1, 0, -1};
    static constexpr int cz[4] = {0, 0, 0, 0};
    static constexpr int opp[4] = {2, 3, 0, 1};
    static constexpr double w0 = 1.0 / 4.0, w1 = 1.0 / 4.0;
    static constexpr double cs2 = 1.0 / 2.0, inv_cs2 = 2.0;
};

struct LatD3Q6 {
    static constexpr int D = 3, Q = 6, NS = 4, A0 = 0, R = 0, K = 5;
    static constexpr bool DIAG = false;
    static constexpr double w[6] = {1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
    static constexpr int wc[6] = {1, 1, 1, 1, 1, 1};
    static constexpr int cx[6] = {1, -1, 0, 0, 0, 0};
    static constexpr int cy[6] = {0, 0, 1, -1, 0, 0};
    static constexpr int cz[6] = {0, 0, 0, 0, 1, -1};
    static constexpr int opp[6] = {1, 0, 3, 2, 5, 4};
    static constexpr double w0 = 1.0 / 6.0, w1 = 1.0 / 6.0;
    static constexpr double cs2 = 1.0 / 3.0, inv_cs2 = 3.0;
};

// D2Q9 (eq. d2q9) and D3Q15 (eq. d3q15), in the printed column order: a
// rest population, axis links and diagonal links with weights of their own
// (w / cs^2 = 1/3 on the axes, 1/12 and 1/24 on the diagonals).
struct LatD2Q9 {
    static constexpr int D = 2, Q = 9, NS = 3, A0 = 0, R = 1, K = 0;
    static constexpr bool DIAG = true;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    static constexpr int wc[9] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    static constexpr double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0;
    static constexpr double cs2 = 1.0 / 3.0, inv_cs2 = 3.0;
};

struct LatD3Q15 {
    static constexpr int D = 3, Q = 15, NS = 4, A0 = 0, R = 1, K = 0;
    static constexpr bool DIAG = true;
    static constexpr int cx[15] = {0, 1, -1, 0, 0, 0, 0, 1, 1, 1, -1, -1, -1, 1, -1};
    static constexpr int cy[15] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, 1, -1, 1, -1, -1};
    static constexpr int cz[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, 1, -1, -1, -1};
    static constexpr int opp[15] = {0, 2, 1, 4, 3, 6, 5, 14, 11, 12, 13, 8, 9, 10, 7};
    static constexpr double w[15] = {2.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0,
                                     1.0 / 72.0, 1.0 / 72.0};
    static constexpr int wc[15] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr double w0 = 2.0 / 9.0, w1 = 1.0 / 9.0;
    static constexpr double cs2 = 1.0 / 3.0, inv_cs2 = 3.0;
};

// The table of opposite directions: c_opp(i) = -c_i for every i, with the
// same weight class (the wall rule and the pair-form collision rely on it).
template <class L>
constexpr bool opposites_ok()
{
    for (int i = 0; i < L::Q; ++i)
        if (L::cx[L::opp[i]] != -L::cx[i] || L::cy[L::opp[i]] != -L::cy[i] || L::cz[L::opp[i]] != -L::cz[i] ||
            L::wc[L::opp[i]] != L::wc[i] || L::w[L::opp[i]] != L::w[i])
            return false;
    return true;
}

// The same lattices storing only the velocity sets a = 1..d.
struct LatD2Q5V : LatD2Q5 {
    static constexpr int NS = 2, A0 = 1;
};
struct LatD3Q7V : LatD3Q7 {
    static constexpr int NS = 3, A0 = 1;
};
struct LatD2Q4V : LatD2Q4 {
    static constexpr int NS = 2, A0 = 1;
};
struct LatD3Q6V : LatD3Q6 {
    static constexpr int NS = 3, A0 = 1;
};
struct LatD2Q9V : LatD2Q9 {
    static constexpr int NS = 2, A0 = 1;
};
struct LatD3Q15V : LatD3Q15 {
    static constexpr int NS = 3, A0 = 1;
};

// A lattice per set (the paper allows a different lattice for each set a,
// remark after eq. d3q15): the velocity sets on D2Q9 / D3Q15, the set a = 0
// on D2Q5 / D3Q7, whose velocities are the first five / seven of the larger
// lattice in the same order (so opposite directions, weight classes and
// link bits carry over).  The set a = 0 only advects rho0, so it can take
// the cheaper lattice: 5 + 2 x 9 planes instead of 27 in 2D, 7 + 3 x 15
// instead of 60 in 3D.  Members Q0, w_set0 and inv_cs2_set0 describe the set
// a = 0.
struct LatD2Q9Q5 : LatD2Q9 {
    static constexpr int Q0 = 5;
    static constexpr double w_set0[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
    static constexpr double inv_cs2_set0 = 3.0;
};
struct LatD3Q15Q7 : LatD3Q15 {
    static constexpr int Q0 = 7;
    static constexpr double w_set0[7] = {1.0 / 4.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0};
    static constexpr double inv_cs2_set0 = 4.0;
};

template <class L, class = void> struct HasSet0Lattice : std::false_type {};
template <class L> struct HasSet0Lattice<L, std::void_t<decltype(L::Q0)>> : std::true_type {};

// Directions, weights and 1/cs^2 of set pa (the set index a of eq. 2-2).
template <class L>
__device__ __forceinline__ constexpr int qset(int pa)
{
    if constexpr (HasSet0Lattice<L>::value) return pa == 0 ? L::Q0 : L::Q;
    else return L::Q;
}
template <class L>
__device__ __forceinline__ constexpr double wset(int pa, int i)
{
    if constexpr (HasSet0Lattice<L>::value) return pa == 0 ? L::w_set0[i < L::Q0 ? i : 0] : L::w[i];
    else return L::w[i];
}
template <class L>
__device__ __forceinline__ constexpr double inv_cs2_set(int pa)
{
    if constexpr (HasSet0Lattice<L>::value) return pa == 0 ? L::inv_cs2_set0 : L::inv_cs2;
    else return L::inv_cs2;
}

// Plane of stored set a, direction i: the sets one after the other, each
// with its own number of directions.
template <class L>
__device__ __host__ __forceinline__ constexpr long long plane_of(int a, int i)
{
    if constexpr (HasSet0Lattice<L>::value) return a == 0 ? i : L::Q0 + (long long)(a - 1) * L::Q + i;
    else return (long long)a * L::Q + i;
}

static_assert(opposites_ok<LatD2Q5>() && opposites_ok<LatD3Q7>() && opposites_ok<LatD2Q4>() &&
                  opposites_ok<LatD3Q6>() && opposites_ok<LatD2Q9>() && opposites_ok<LatD3Q15>(),
              "opposite-direction tables");

template <class L>
__device__ __forceinline__ constexpr int cdir(int i, int b)
{
    return b == 0 ? L::cx[i] : (b == 1 ? L::cy[i] : L::cz[i]);
}

// ----------------------------------------------------------------- tiling

// Tile handled by this block.  Workgroups of a 1D grid are dealt to the
// XCDs round-robin (block b runs on XCD b % groups); with groups > 1 the
// tiles are renumbered so that each XCD receives one contiguous band of
// tiles, so that the x- and y-neighbours a tile's pulls straddle into sit in
// the same L2.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ int block_tile(const Tiling &t)
{
    const int b = blockIdx.x;
    if (t.groups <= 1) return b;
    const int q = t.nb / t.groups, r = t.nb % t.groups;
    const int g = b % t.groups, k = b / t.groups;
    return (g < r) ? g * (q + 1) + k : r * (q + 1) + (g - r) * q + k;
}

// ----------------------------------------------------------------- storage

// Storage codes follow mdf_storage.  decode/encode convert one stored value;
// load/store address it.  VX is the number of consecutive x-nodes one thread
// owns in the vector step kernel: one 16-byte access per plane for FP64 and
// FP32, 8 bytes for the 16-bit formats.
template <int ST> struct Store;

// A node's place in a plane is an element index: 64-bit in general, or an
// Ix32 when every population plane and field channel of the launch spans at
// most 4 GiB.  With an Ix32 the address of an access is the plane's base,
// the same for the whole wavefront (scalar registers), plus a 32-bit byte
// offset that the load or store adds itself; a 64-bit index costs two
// 64-bit vector operations per plane and node instead.
struct Ix32 {
    uint32_t k;
};

template <class T>
__device__ __forceinline__ T *elem(T *p, long long k)
{
    return p + k;
}

// Element i of the plane at p, a global-memory address that every lane of
// the wavefront passes alike.  The base goes through readfirstlane: the
// opaque copy keeps the optimizer from folding the per-plane part of the
// address into one shared 64-bit vector address, which would bring the
// 64-bit vector arithmetic back.
template <class T>
__device__ __forceinline__ T *elem(T *p, Ix32 i)
{
    using G = __attribute__((address_space(1))) char;   // global memory
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint64_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint64_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
    G *g = (G *)(hi << 32 | lo);
    return (T *)(g + i.k * uint32_t(sizeof(T)));
}

// Index of node (x, y, z) in planes of rows of `pitch` values, ny rows per
// z-slab.
template <bool WIDE>
__device__ __forceinline__ auto grid_ix(int x, int y, int z, int ny, int pitch)
{
    if constexpr (WIDE)
        return ((long long)z * ny + y) * pitch + x;
    else
        return Ix32{(uint32_t(z) * uint32_t(ny) + uint32_t(y)) * uint32_t(pitch) + uint32_t(x)};
}

// One stored value, written with a non-temporal hint when NT: populations
// that the next launch will not find in the 256 MB Infinity Cache anyway skip
// it, which leaves L2 and the cache to the halo and neighbour reads.  On
// working sets that fit the cache the plain store keeps them there for the
// next launch.  NT is a template parameter all the way down: with a run-time
// flag the optimizer merges the two stores of the same value before
// inlining and drops the hint.
template <bool NT, class T, class IX>
__device__ __forceinline__ void put_value(T *p, IX k, T x)
{
    T *q = elem(p, k);
    if constexpr (NT) __builtin_nontemporal_store(x, q);
    else *q = x;
}

template <> struct Store<MDF_F64> {
    using T = double;
    using C = double;
    static constexpr int VX = 2;
    static __device__ __forceinline__ C decode(T v, C, float) { return v; }
    static __device__ __forceinline__ T encode(C v, C, float) { return v; }
    template <class IX>
    static __device__ __forceinline__ C load(const T *p, IX k, C, float) { return *elem(p, k); }
    template <class IX>
    static __device__ __forceinline__ void store(T *p, IX k, C v, C, float) { *elem(p, k) = v; }
    template <bool NT, class IX>
    static __device__ __forceinline__ void store_hint(T *p, IX k, C v, C, float)
    {
        put_value<NT>(p, k, v);
    }
};

template <> struct Store<MDF_F32> {
    using T = float;
    using C = float;
    static constexpr int VX = 4;
    static __device__ __forceinline__ C decode(T v, C, float) { return v; }
    static __device__ __forceinline__ T encode(C v, C, float) { return v; }
    template <class IX>
    static __device__ __forceinline__ C load(const T *p, IX k, C, float) { return *elem(p, k); }
    template <class IX>
    static __device__ __forceinline__ void store(T *p, IX k, C v, C, float) { *elem(p, k) = v; }
    template <bool NT, class IX>
    static __device__ __forceinline__ void store_hint(T *p, IX k, C v, C, float)
    {
        put_value<NT>(p, k, v);
    }
};

// 16-bit deviation storage: stored = (f - rest) / scale, round to nearest even.
template <> struct Store<MDF_F16DEV> {
    using T = _Float16;
    using C = float;
    static constexpr int VX = 4;
    static __device__ __forceinline__ C decode(T v, C rest, float scale)
    {
        return rest + scale * static_cast<float>(v);
    }
    static __device__ __forceinline__ T encode(C v, C rest, float inv_scale)
    {
        return static_cast<_Float16>((v - rest) * inv_scale);
    }
    template <class IX>
    static __device__ __forceinline__ C load(const T *p, IX k, C rest, float scale)
    {
        return decode(*elem(p, k), rest, scale);
    }
    template <class IX>
    static __device__ __forceinline__ void store(T *p, IX k, C v, C rest, float inv_scale)
    {
        *elem(p, k) = encode(v, rest, inv_scale);
    }
    template <bool NT, class IX>
    static __device__ __forceinline__ void store_hint(T *p, IX k, C v, C rest, float inv_scale)
    {
        put_value<NT>(p, k, encode(v, rest, inv_scale));
    }
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <> struct Store<MDF_BF16DEV> {
    using T = uint16_t;
    using C = float;
    static constexpr int VX = 4;
    static __device__ __forceinline__ C decode(T v, C rest, float scale)
    {
        return rest + scale * __uint_as_float(((uint32_t)v) << 16);
    }
    static __device__ __forceinline__ T encode(C v, C rest, float inv_scale)
    {
        return f32_to_bf16_rne((v - rest) * inv_scale);
    }
    template <class IX>
    static __device__ __forceinline__ C load(const T *p, IX k, C rest, float scale)
    {
        return decode(*elem(p, k), rest, scale);
    }
    template <class IX>
    static __device__ __forceinline__ void store(T *p, IX k, C v, C rest, float inv_scale)
    {
        *elem(p, k) = encode(v, rest, inv_scale);
    }
    template <bool NT, class IX>
    static __device__ __forceinline__ void store_hint(T *p, IX k, C v, C rest, float inv_scale)
    {
        put_value<NT>(p, k, encode(v, rest, inv_scale));
    }
};

// VX consecutive stored values, accessed as one aligned vector.
template <class T, int VX>
struct alignas(sizeof(T) * VX) VecT {
    T v[VX];
};

// Raw bits of a vector, as one 8- or 16-byte register tuple, so that a
// vector is moved by exactly one load or store instruction.
template <int B> struct RawVec;
template <> struct RawVec<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct RawVec<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };

template <class T, int VX>
__device__ __forceinline__ VecT<T, VX> vload(const T *p)
{
    using R = typename RawVec<sizeof(T) * VX>::type;
    const R r = *reinterpret_cast<const R *>(p);
    VecT<T, VX> v;
    __builtin_memcpy(&v, &r, sizeof v);
    return v;
}

template <class T, int VX>
__device__ __forceinline__ void vstore(T *p, const VecT<T, VX> &v)
{
    using R = typename RawVec<sizeof(T) * VX>::type;
    R r;
    __builtin_memcpy(&r, &v, sizeof r);
    *reinterpret_cast<R *>(p) = r;
}

// A case parameter in the compute type: the FP32 copy rounded on the host
// for the FP32 and 16-bit kernels, the FP64 value for the FP64 kernels.
template <class C> __device__ __forceinline__ C kpar(double d, float f);
template <> __device__ __forceinline__ float kpar<float>(double, float f) { return f; }
template <> __device__ __forceinline__ double kpar<double>(double d, float) { return d; }

// Value of the lane one below / one above in the wavefront (all lanes must
// execute these; a lane at the wave's edge gets its own value back).
template <class T>
__device__ __forceinline__ T lane_up1(T v)
{
    if constexpr (sizeof(T) == 2) {
        uint16_t b;
        __builtin_memcpy(&b, &v, 2);
        const int r = __shfl_up((int)b, 1, 64);
        const uint16_t o = (uint16_t)r;
        T out;
        __builtin_memcpy(&out, &o, 2);
        return out;
    } else {
        return __shfl_up(v, 1, 64);
    }
}

template <class T>
__device__ __forceinline__ T lane_down1(T v)
{
    if constexpr (sizeof(T) == 2) {
        uint16_t b;
        __builtin_memcpy(&b, &v, 2);
        const int r = __shfl_down((int)b, 1, 64);
        const uint16_t o = (uint16_t)r;
        T out;
        __builtin_memcpy(&out, &o, 2);
        return out;
    } else {
        return __shfl_down(v, 1, 64);
    }
}

// rest state of a population: w_i rho0 for the set a = 0, zero otherwise
// (pressure gauge P = 0).
template <class L, class C>
__device__ __forceinline__ C rest_value(const KCase &p, int a, int i)
{
    if (a + L::A0 != 0) return C(0);
    return kpar<C>(p.restd[L::wc[i]], p.restf[L::wc[i]]);
}

// ----------------------------------------------------------------- node state

template <class L, class C>
struct Node {
    C f[L::NS][L::Q];       // pre-collision populations f(x, t)
    C fb[L::D + 1];         // source Fbar_a of every set at the node (read with the populations)
};

template <class L, class C>
struct Moments {
    C ubar[L::D + 1];       // eq. 2-7, sets a = 0..d (a = 0: rho0 when that set is not stored)
    C u[L::D];
    C P;                    // eq. 3-15
    C trJ;                  // sum_{a>=1} J_{a,a}
    C fb[L::D + 1];         // Fbar_a at the node: uniform part + force field
};

// Source Fbar_a of set a at a node (eq. 2-2, eq. 2-6): Fbar_0 = R, Fbar_a =
// the uniform force plus the per-node force field when one is set.
template <class C>
__device__ __forceinline__ C source_of(const KCase &p, int pa, long long node)
{
    C fb = kpar<C>(p.fbar[pa], p.fbarf[pa]);
    if (pa >= 1 && p.ffield)
        fb += static_cast<const C *>(p.ffield)[(long long)(pa - 1) * ((long long)p.nx * p.ny * p.nz) + node];
    return fb;
}

// The sources of every set at a node.  Issued together with the node's
// population loads, so that a force field's loads do not wait behind them.
template <class L, class C>
__device__ __forceinline__ void load_sources(const KCase &p, long long node, Node<L, C> &n)
{
#pragma unroll
    for (int pa = 0; pa <= L::D; ++pa) n.fb[pa] = source_of<C>(p, pa, node);
}

// Wall face a pull of direction i at node (x, y, z) crosses: 0..5 for a
// wall face, 6 for a solid upstream node (MASK), -1 for a plain pull, whose
// upstream node (wrapped across periodic faces) is returned in sx, sy, sz.
// With PULL = false the node reads its own values: no face, (sx, sy, sz) =
// (x, y, z).
template <class L, bool MASK, bool PULL, bool WIDE>
__device__ __forceinline__ int pull_face(const KCase &p, const uint8_t *__restrict__ links, unsigned lb, int x,
                                         int y, int z, int i, int &sx, int &sy, int &sz)
{
    sx = x - L::cx[i];
    sy = y - L::cy[i];
    sz = z - L::cz[i];
    if (!PULL) {
        sx = x; sy = y; sz = z;
        return -1;
    }
    int face = -1;
    if (L::cx[i] != 0) {
        if (sx < 0) { if (p.bc[0] == MDF_WALL) face = 0; else sx += p.nx; }
        else if (sx >= p.nx) { if (p.bc[1] == MDF_WALL) face = 1; else sx -= p.nx; }
    }
    if (L::cy[i] != 0) {
        if (sy < 0) { if (p.bc[2] == MDF_WALL) { if (face < 0) face = 2; } else sy += p.ny; }
        else if (sy >= p.ny) { if (p.bc[3] == MDF_WALL) { if (face < 0) face = 3; } else sy -= p.ny; }
    }
    if (L::cz[i] != 0) {
        if (sz < 0) { if (p.bc[4] == MDF_WALL) { if (face < 0) face = 4; } else sz += p.nz; }
        else if (sz >= p.nz) { if (p.bc[5] == MDF_WALL) { if (face < 0) face = 5; } else sz -= p.nz; }
    }
    if (MASK && face < 0) {
        if constexpr (L::DIAG) {
            // more moving directions than link bits: read the upstream
            // node's solid flag
            if (*elem(links, grid_ix<WIDE>(sx, sy, sz, p.ny, p.pitch)) & 0x80u) face = 6;
        } else if ((lb >> i) & 1u) {
            face = 6;
        }
    }
    return face;
}

// A node's pull in the 16-bit formats, in two parts: gather_issue() issues
// every population load (and finds the wall faces), gather_decode() decodes
// and applies the wall rule.  A decode right after each load makes the node
// wait for its loads one direction at a time (measured: 2.6x on the 3D
// two-step kernel, +11 % on the 2D one).  (Issuing the loads of all of a
// thread's nodes in a tile kernel before decoding any measured the same in
// 2D and left the 3D two-step kernel with phi values of undefined 16-bit
// loads, which the compiler folded to NaN constants: 250 extra moves.)
template <class L, int ST>
struct Pulled {
    typename Store<ST>::T raw[L::NS][L::Q];
    int fc[L::Q];
};

template <class L, int ST, bool MASK, bool PULL, bool WIDE = true>
__device__ __forceinline__ bool gather_issue(const KCase &p, const typename Store<ST>::T *__restrict__ src,
                                             const uint8_t *__restrict__ links, int x, int y, int z,
                                             Node<L, typename Store<ST>::C> &n, Pulled<L, ST> &r)
{
    using C = typename Store<ST>::C;
    const auto own = grid_ix<WIDE>(x, y, z, p.ny, p.pitch);
    unsigned lb = 0;
    if (MASK) {
        lb = *elem(links, own);
        if (lb & 0x80u) return false;
    }
    load_sources<L, C>(p, ((long long)z * p.ny + y) * p.nx + x, n);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int sx, sy, sz;
        const int face = pull_face<L, MASK, PULL, WIDE>(p, links, lb, x, y, z, i, sx, sy, sz);
        r.fc[i] = face;
        if constexpr (!WIDE) {
            // every lane reads plane i, at the upstream node or (a wall or a
            // solid link; re-read below) at its own: one
            // 32-bit offset per direction with each plane's scalar base, for
            // every set.  The empty asm keeps the optimizer from widening the
            // per-lane choice to a 64-bit address select.
            uint32_t k = (face < 0) ? grid_ix<false>(sx, sy, sz, p.ny, p.pitch).k : own.k;
            asm volatile("" : "+v"(k));
#pragma unroll
            for (int a = 0; a < L::NS; ++a)
                if (i < qset<L>(a + L::A0)) r.raw[a][i] = *elem(src + plane_of<L>(a, i) * p.dstride, Ix32{k});
        } else if (face < 0) {
            const auto k = grid_ix<WIDE>(sx, sy, sz, p.ny, p.pitch);
#pragma unroll
            for (int a = 0; a < L::NS; ++a)
                if (i < qset<L>(a + L::A0)) r.raw[a][i] = *elem(src + plane_of<L>(a, i) * p.dstride, k);
        } else {
            const int j = L::opp[i];
#pragma unroll
            for (int a = 0; a < L::NS; ++a)
                if (i < qset<L>(a + L::A0)) r.raw[a][i] = *elem(src + plane_of<L>(a, j) * p.dstride, own);
        }
    }
    if constexpr (!WIDE) {
        // the lanes that pulled across a wall or from a solid node read the
        // opposite direction at their own node, in a branch that interior
        // wavefronts skip
        bool wall = false;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) wall |= r.fc[i] >= 0;
        if (__builtin_amdgcn_ballot_w64(wall) != 0) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                if (r.fc[i] < 0) continue;
                const int j = L::opp[i];
#pragma unroll
                for (int a = 0; a < L::NS; ++a)
                    if (i < qset<L>(a + L::A0)) r.raw[a][i] = *elem(src + plane_of<L>(a, j) * p.dstride, own);
            }
        }
    }
    return true;
}

template <class L, int ST>
__device__ __forceinline__ void gather_decode(const KCase &p, const Pulled<L, ST> &r,
                                              Node<L, typename Store<ST>::C> &n)
{
    using S = Store<ST>;
    using C = typename S::C;
    // (a direction and its opposite share their weight class, hence their
    // rest value)
    bool wall = false;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        wall |= r.fc[i] >= 0;
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            if (i >= qset<L>(a + L::A0)) { n.f[a][i] = C(0); continue; }
            n.f[a][i] = S::decode(r.raw[a][i], rest_value<L, C>(p, a, i), p.scale);
        }
    }
    // The wall rule on the velocity sets, only in a wavefront where some
    // lane pulled across a wall or from a solid node: a uniform branch that
    // interior wavefronts skip (as selects it cost every node about five
    // vector instructions per velocity-set population).
    if (__builtin_amdgcn_ballot_w64(wall) != 0) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (r.fc[i] < 0) continue;
            const C w = C(L::w[i]);
#pragma unroll
            for (int a = 0; a < L::NS; ++a) {
                if (a + L::A0 == 0 || i >= qset<L>(a + L::A0)) continue;
                const int b = a + L::A0 - 1;
                // the face's wall velocity, selected with constant indices (a
                // run-time index into the case parameters here copied them to
                // scratch memory)
                C uw = C(0);
#pragma unroll
                for (int f = 0; f < 6; ++f)
                    if (r.fc[i] == f) uw = kpar<C>(p.wallu[f][b], p.walluf[f][b]);
                const C v = n.f[a][i];
                n.f[a][i] = -v + C(2) * w * uw;
            }
        }
    }
}

// The storages whose pulls go through gather_issue() / gather_decode().
template <int ST>
constexpr bool kSplitPull = sizeof(typename Store<ST>::T) == 2;

// Pull the populations of node (x, y, z) at time t+1 out of the
// post-collision planes of time t (or, with PULL = false, read the node's
// own stored pre-collision values).  Returns false for a solid node.
// FP32 and FP64 values need no decode and are pulled in a single pass, which
// holds fewer registers.
template <class L, int ST, bool MASK, bool PULL, bool WIDE = true>
__device__ __forceinline__ bool gather(const KCase &p, const typename Store<ST>::T *__restrict__ src,
                                       const uint8_t *__restrict__ links, int x, int y, int z,
                                       Node<L, typename Store<ST>::C> &n)
{
    using S = Store<ST>;
    using C = typename S::C;
    if constexpr (kSplitPull<ST>) {
        Pulled<L, ST> r;
        if (!gather_issue<L, ST, MASK, PULL, WIDE>(p, src, links, x, y, z, n, r)) return false;
        gather_decode<L, ST>(p, r, n);
        return true;
    } else {
        const auto own = grid_ix<WIDE>(x, y, z, p.ny, p.pitch);
        unsigned lb = 0;
        if (MASK) {
            lb = *elem(links, own);
            if (lb & 0x80u) return false;
        }
        load_sources<L, C>(p, ((long long)z * p.ny + y) * p.nx + x, n);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            int sx, sy, sz;
            const int face = pull_face<L, MASK, PULL, WIDE>(p, links, lb, x, y, z, i, sx, sy, sz);
            const C w = C(L::w[i]);
            if (face < 0) {
                const auto k = grid_ix<WIDE>(sx, sy, sz, p.ny, p.pitch);
#pragma unroll
                for (int a = 0; a < L::NS; ++a) {
                    if (i >= qset<L>(a + L::A0)) { n.f[a][i] = C(0); continue; }
                    n.f[a][i] = S::load(src + plane_of<L>(a, i) * p.dstride, k, rest_value<L, C>(p, a, i), p.scale);
                }
            } else {
                const int j = L::opp[i];
#pragma unroll
                for (int a = 0; a < L::NS; ++a) {
                    if (i >= qset<L>(a + L::A0)) { n.f[a][i] = C(0); continue; }
                    C v = S::load(src + plane_of<L>(a, j) * p.dstride, own, rest_value<L, C>(p, a, j), p.scale);
                    if (a + L::A0 == 0) {
                        n.f[a][i] = v;
                    } else {
                        const int b = a + L::A0 - 1;
                        C uw = (face < 6) ? kpar<C>(p.wallu[face][b], p.walluf[face][b]) : C(0);
                        n.f[a][i] = -v + C(2) * w * uw;
                    }
                }
            }
        }
        return true;
    }
}

// Vector form of gather(): the thread owns the VX consecutive nodes
// x0 .. x0+VX-1 of row (y, z) (x0 a multiple of VX, rows padded to whole
// 128-byte lines, so every vector lies inside its padded row).  Each plane
// is read as one aligned vector per thread: for directions with c_x = 0 from
// the upstream row, for c_x = +-1 from the own row, the one value the shift
// pulls in from outside the vector coming from the neighbouring lane (or, at
// the edge of a wavefront or a tile row, from one scalar load).  Periodic
// wraps in x, walls and solid links are resolved per node with scalar loads
// (the same values gather() reads).  Every lane must call this (it
// exchanges values between lanes); `rowok` says whether the thread owns any
// node, `fix_lo` / `fix_hi` whether its lower / upper neighbour in x lies
// in another wavefront or tile row.
template <class L, int ST, bool MASK, int VX>
__device__ __forceinline__ void gather_vec(const KCase &p, const typename Store<ST>::T *__restrict__ src,
                                           const uint8_t *__restrict__ links, int x0, int y, int z, bool rowok,
                                           bool fix_lo, bool fix_hi, Node<L, typename Store<ST>::C> (&n)[VX],
                                           bool (&fluid)[VX])
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    const long long own = ((long long)z * p.ny + y) * p.pitch + x0;
    unsigned lb[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const bool in = rowok && (x0 + v < p.nx);
        lb[v] = (MASK && in) ? links[own + v] : 0u;
        fluid[v] = in && !(lb[v] & 0x80u);
        if (in) load_sources<L, C>(p, ((long long)z * p.ny + y) * p.nx + x0 + v, n[v]);
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int cxi = L::cx[i];
        int sy = y - L::cy[i], sz = z - L::cz[i];
        int face = -1;
        if (L::cy[i] != 0) {
            if (sy < 0) { if (p.bc[2] == MDF_WALL) { if (face < 0) face = 2; } else sy += p.ny; }
            else if (sy >= p.ny) { if (p.bc[3] == MDF_WALL) { if (face < 0) face = 3; } else sy -= p.ny; }
        }
        if (L::cz[i] != 0) {
            if (sz < 0) { if (p.bc[4] == MDF_WALL) { if (face < 0) face = 4; } else sz += p.nz; }
            else if (sz >= p.nz) { if (p.bc[5] == MDF_WALL) { if (face < 0) face = 5; } else sz -= p.nz; }
        }
        const C w = C(L::w[i]);
        const int j = L::opp[i];
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            const T *plane = src + plane_of<L>(a, i) * p.dstride;
            const T *oplane = src + plane_of<L>(a, j) * p.dstride;
            const C rest_i = rest_value<L, C>(p, a, i), rest_j = rest_value<L, C>(p, a, j);
            VecT<T, VX> vec;
#pragma unroll
            for (int v = 0; v < VX; ++v) vec.v[v] = T(0);
            if (rowok && face < 0) vec = vload<T, VX>(plane + ((long long)sz * p.ny + sy) * p.pitch + x0);
            T lo = T(0), hi = T(0);
            if (cxi > 0) {
                lo = lane_up1(vec.v[VX - 1]);
                if (rowok && fix_lo && x0 > 0) lo = plane[own - 1];
            }
            if (cxi < 0) {
                hi = lane_down1(vec.v[0]);
                if (rowok && fix_hi && x0 + VX < p.nx) hi = plane[own + VX];
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                if (!fluid[v]) continue;
                int sx = x0 + v - cxi;
                int f = face;
                bool wrapped = false;
                if (cxi != 0) {
                    if (sx < 0) { if (p.bc[0] == MDF_WALL) f = 0; else { sx += p.nx; wrapped = true; } }
                    else if (sx >= p.nx) { if (p.bc[1] == MDF_WALL) f = 1; else { sx -= p.nx; wrapped = true; } }
                }
                if (MASK && f < 0 && ((lb[v] >> i) & 1u)) f = 6;
                if (f >= 0) {
                    const C val = S::decode(oplane[own + v], rest_j, p.scale);
                    if (a + L::A0 == 0) {
                        n[v].f[a][i] = val;
                    } else {
                        const int b = a + L::A0 - 1;
                        const C uw = (f < 6) ? kpar<C>(p.wallu[f][b], p.walluf[f][b]) : C(0);
                        n[v].f[a][i] = -val + C(2) * w * uw;
                    }
                } else {
                    T raw;
                    const int k = v - cxi;
                    if (wrapped) raw = plane[own - x0 + sx];
                    else if (k < 0) raw = lo;
                    else if (k >= VX) raw = hi;
                    else raw = vec.v[k < 0 ? 0 : (k >= VX ? VX - 1 : k)];
                    n[v].f[a][i] = S::decode(raw, rest_i, p.scale);
                }
            }
        }
    }
}

// eq. 2-7 (Scheme II: eq. 2-7a) and eq. 3-15, and the source of every set.
template <class L, class C>
__device__ __forceinline__ void moments(const KCase &p, const Node<L, C> &n, Moments<L, C> &m)
{
#pragma unroll
    for (int pa = 0; pa <= L::D; ++pa) m.fb[pa] = n.fb[pa];
#pragma unroll
    for (int a = 0; a < L::NS; ++a) {
        C s = n.f[a][0];
#pragma unroll
        for (int i = 1; i < L::Q; ++i) s += n.f[a][i];
        // Scheme II stores fbar = f - F/2: half the source is added back
        if (p.forcing == MDF_FORCING_SCHEME2) s += C(0.5) * m.fb[a + L::A0];
        m.ubar[a + L::A0] = s;
    }
    if (L::A0 == 1) m.ubar[0] = kpar<C>(p.rho0, p.rho0f);
#pragma unroll
    for (int b = 0; b < L::D; ++b) m.u[b] = m.ubar[b + 1];
    C trJ = C(0), u2 = C(0);
#pragma unroll
    for (int pa = 1; pa <= L::D; ++pa) {     // velocity sets
        const int a = pa - L::A0;
        C j = C(0);
#pragma unroll
        for (int i = L::R; i < L::Q; ++i) {
            if (cdir<L>(i, pa - 1) > 0) j += n.f[a][i];
            else if (cdir<L>(i, pa - 1) < 0) j -= n.f[a][i];
        }
        trJ += j;
        u2 += m.u[pa - 1] * m.u[pa - 1];
    }
    m.trJ = trJ;
    m.P = (trJ + kpar<C>(p.rps, p.rpsf) - u2) * C(1.0 / L::D);
}

// Equilibrium of one set (eq. 2-4), f^eq_i = w_i [ubar + c_i . flux / cs^2]
// with flux = ubar u + P E_a, evaluated in a form that is exact in any
// precision where the weights are not: w_i / cs^2 is 1/2 for every moving
// population of D2Q5 and D3Q7, and the rest weight is taken as
// w_0 = 1 - sum_{i>0} w_i, so
// f^eq_0 = ubar - sum_{i>0} w_i ubar.  (With w_0 = 1/3 and w_1 = 1/6 rounded
// to FP32, sum_i w_i differs from 1 by ~3e-8, and the zeroth moment would
// drift by that fraction every step.)  Without a rest population the
// collision closes the zeroth moment instead (collide_fused()).
template <class L, class C>
__device__ __forceinline__ void equilibrium(C ub, const C (&flux)[L::D], C (&feq)[L::Q], int pa)
{
    C rest = ub;
#pragma unroll
    for (int i = L::R; i < L::Q; ++i) {
        if (i >= qset<L>(pa)) { feq[i] = C(0); continue; }
        C cf = C(0);
#pragma unroll
        for (int b = 0; b < L::D; ++b) {
            if (cdir<L>(i, b) > 0) cf += flux[b];
            else if (cdir<L>(i, b) < 0) cf -= flux[b];
        }
        const C even = C(wset<L>(pa, i)) * ub;
        feq[i] = even + C(wset<L>(pa, i) * inv_cs2_set<L>(pa)) * cf;
        rest -= even;
    }
    if (L::R == 1) feq[0] = rest;
}

// Non-equilibrium part n_{i,a} = f_{i,a} - f^eq_{i,a} of one set.
template <class L, class C>
__device__ __forceinline__ void nonequilibrium(const Node<L, C> &n, const Moments<L, C> &m, int a,
                                               C (&ne)[L::Q])
{
    const int pa = a + L::A0;              // set index a of the stored set
    const C ub = m.ubar[pa];
    C flux[L::D];
#pragma unroll
    for (int b = 0; b < L::D; ++b) flux[b] = ub * m.u[b] + ((pa >= 1 && b == pa - 1) ? m.P : C(0));
    C feq[L::Q];
    equilibrium<L, C>(ub, flux, feq, pa);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) ne[i] = n.f[a][i] - feq[i];
}

// Post-collision populations of one set (right-hand side of eq. 3-21, or of
// eq. 2-3c under Scheme II).
// The s0 part of L n multiplies sum_i n_i, which vanishes identically
// (eq. 3-8); the moving populations take s1 on the odd and s2 on the even part
// of n.  Each population is advanced by a small increment d_i computed first,
// f*_i = f_i + d_i, and the rest population takes d_0 = Fbar - sum_{i>0} d_i,
// which is the zeroth-moment identity sum_i f*_i = ubar + Fbar (eq. 3-9 with
// eq. 3-7c).  In exact arithmetic this is the matrix product; in FP32 every
// stored value is rounded once, and the zeroth moment is conserved up to
// unbiased rounding (forming s0 sum_i n_i, or subtracting large partial sums,
// rounds the same way every step and drifts by ~1e-5 in a few thousand).
// Scheme II: with n = fbar - f^eq (ubar from eq. 2-7a), the update is
// fbar + F - L (n + F/2), and sum_i (n + F/2)_i = 0, so the same projection
// applies; F/2 is even, which turns the force on the moving populations
// into (1 - s2/2) w_i Fbar while sum_i fbar*_i = ubar - Fbar/2 + Fbar still
// fixes the rest population.  On lattices without a rest population the
// last moving population K takes that identity in the same way: in exact
// arithmetic its value is unchanged, and in FP32 the zeroth moment does not
// inherit the rounding of w = 1/6 (D3Q6) every step.
// The update is taken per pair of opposite directions (i, j = opp(i)), which
// share their weight and the even part of the equilibrium and have opposite
// odd parts:
//   f^eq_{i,j} = w ubar +- (w / cs^2) c_i . flux                     (eq. 2-4)
//   n_i - n_j = (f_i - f_j) - 2 (w / cs^2) c_i . flux  (odd part of n)
//   n_i + n_j = (f_i + f_j) - 2 w ubar                 (even part of n)
//   d_{i,j} = w Fbar' - (s2/2)(n_i + n_j) -+ (s1/2)(n_i - n_j)
// (Fbar' = Fbar, or (1 - s2/2) Fbar under Scheme II), and the rest
// population (or K) closes the zeroth moment as above.  The equilibrium is
// never formed per population, which halves the arithmetic of forming f^eq,
// n = f - f^eq and the relaxation one population at a time.
template <class L, class C>
__device__ __forceinline__ void collide_fused(const KCase &p, const Node<L, C> &n, const Moments<L, C> &m, int a,
                                              C (&out)[L::Q], C fb)
{
    const int pa = a + L::A0;
    const C ub = m.ubar[pa];
    C flux[L::D];
#pragma unroll
    for (int b = 0; b < L::D; ++b) flux[b] = ub * m.u[b] + ((pa >= 1 && b == pa - 1) ? m.P : C(0));
    const C s1h = C(0.5) * kpar<C>(p.s1, p.s1f), s2h = C(0.5) * kpar<C>(p.s2, p.s2f);
    const C fm = fb * kpar<C>(p.fmove, p.fmovef);
    C dsum = C(0);
#pragma unroll
    for (int i = L::R; i < L::Q; ++i) {
        const int j = L::opp[i];
        if (j < i) continue;                       // each pair once
        if (i >= qset<L>(pa)) { out[i] = C(0); out[j] = C(0); continue; }
        C cf = C(0);
#pragma unroll
        for (int b = 0; b < L::D; ++b) {
            if (cdir<L>(i, b) > 0) cf += flux[b];
            else if (cdir<L>(i, b) < 0) cf -= flux[b];
        }
        const C w = C(wset<L>(pa, i));
        const C odd2 = C(2.0 * wset<L>(pa, i) * inv_cs2_set<L>(pa)) * cf;     // 2 (w / cs^2) c_i . flux
        const C even2 = C(2) * w * ub;                                        // 2 w ubar
        const C nodd = (n.f[a][i] - n.f[a][j]) - odd2;
        const C neven = (n.f[a][i] + n.f[a][j]) - even2;
        const C base = w * fm - s2h * neven;
        const C di = base - s1h * nodd, dj = base + s1h * nodd;
        if (i != L::K) { out[i] = n.f[a][i] + di; dsum += di; }
        if (j != L::K) { out[j] = n.f[a][j] + dj; dsum += dj; }
    }
    out[L::K] = n.f[a][L::K] + (fb - dsum);
}

// Channels of the field selection `fields` (order of the MDF_FIELD_* bits).
template <class L>
__device__ __forceinline__ int field_channels(uint32_t fields)
{
    int nch = 0;
    if (fields & MDF_FIELD_MOMENTS) nch += L::D + 2;
    if (fields & MDF_FIELD_GRAD) nch += L::D * L::D;
    if (fields & MDF_FIELD_DIV) nch += 1;
    if (fields & MDF_FIELD_STRAIN) nch += L::D * (L::D + 1) / 2;
    if (fields & MDF_FIELD_STRESS) nch += L::D * (L::D + 1) / 2;
    if (fields & MDF_FIELD_VORT) nch += (L::D == 2 ? 1 : 3);
    return nch;
}

// One emitted value: written, or (MDF_FIELD_ACCUMULATE) added to what the
// channel holds.
template <class C, class IX>
__device__ __forceinline__ void emit_value(C *ch, IX node, C v, bool acc)
{
    if (acc) v += *elem(ch, node);
    put_value<false>(ch, node, v);
}

// A solid node emits zero in every selected channel (adds nothing when
// accumulating).
template <class L, class C, class IX>
__device__ __forceinline__ void write_zero_fields(uint32_t fields, C *__restrict__ out, IX node, long long nodes)
{
    if (fields & MDF_FIELD_ACCUMULATE) return;
    const int nch = field_channels<L>(fields);
    for (int ch = 0; ch < nch; ++ch) put_value<false>(out + ch * nodes, node, C(0));
}

// Derived fields of eq. 3-16..3-19 written channel-major for the selection
// `fields` (order of the MDF_FIELD_* bits).
template <class L, class C, class IX>
__device__ __forceinline__ void write_fields(const KCase &p, const Node<L, C> &n,
                                             const Moments<L, C> &m, uint32_t fields, C *__restrict__ out,
                                             IX node, long long nodes)
{
    constexpr int D = L::D;
    // first moment of the non-equilibrium part, mne[a][b] = sum_i c_{i,b} n_{i,a}
    C mne[D][D];
#pragma unroll
    for (int pa = 1; pa <= D; ++pa) {       // velocity sets
        C ne[L::Q];
        nonequilibrium<L, C>(n, m, pa - L::A0, ne);
#pragma unroll
        for (int b = 0; b < D; ++b) {
            C s = C(0);
#pragma unroll
            for (int i = L::R; i < L::Q; ++i) {
                if (cdir<L>(i, b) > 0) s += ne[i];
                else if (cdir<L>(i, b) < 0) s -= ne[i];
            }
            mne[pa - 1][b] = s;
        }
    }
    const C gscale = -kpar<C>(p.s1, p.s1f) * C(L::inv_cs2);           // eq. 3-16
    C G[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) G[a][b] = gscale * mne[a][b];
    const bool acc = (fields & MDF_FIELD_ACCUMULATE) != 0;
    long long ch = 0;
    if (fields & MDF_FIELD_MOMENTS) {
#pragma unroll
        for (int a = 0; a <= L::D; ++a) emit_value(out + (ch++) * nodes, node, m.ubar[a], acc);
        emit_value(out + (ch++) * nodes, node, m.P, acc);
    }
    if (fields & MDF_FIELD_GRAD) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) emit_value(out + (ch++) * nodes, node, G[a][b], acc);
    }
    if (fields & MDF_FIELD_DIV) {
        C dv = G[0][0];
#pragma unroll
        for (int a = 1; a < D; ++a) dv += G[a][a];
        emit_value(out + (ch++) * nodes, node, dv, acc);                  // eq. 3-16a
    }
    if (fields & MDF_FIELD_STRAIN) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                emit_value(out + (ch++) * nodes, node, C(0.5) * (G[a][b] + G[b][a]), acc);   // eq. 3-17
    }
    if (fields & MDF_FIELD_STRESS) {
        const C sc = -kpar<C>(p.rho0, p.rho0f) * (C(1) - C(0.5) * kpar<C>(p.s1, p.s1f));   // eq. 3-17a
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                emit_value(out + (ch++) * nodes, node, sc * (mne[a][b] + mne[b][a]), acc);
    }
    if (fields & MDF_FIELD_VORT) {
        // omega = curl u; Omega_ab = (G_ab - G_ba)/2 (eq. 3-18) and
        // Omega_ab = -eps_abg omega_g / 2 (eq. 3-19)
        if (D == 2) {
            emit_value(out + (ch++) * nodes, node, G[1][0] - G[0][1], acc);
        } else {
            emit_value(out + (ch++) * nodes, node, G[2 % D][1 % D] - G[1 % D][2 % D], acc);
            emit_value(out + (ch++) * nodes, node, G[0][2 % D] - G[2 % D][0], acc);
            emit_value(out + (ch++) * nodes, node, G[1 % D][0] - G[0][1 % D], acc);
        }
    }
}

// ----------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block reduction of kNRed doubles into partial[tile].
__device__ __forceinline__ void block_reduce_store(double (&v)[kNRed], double *__restrict__ partial, int tile)
{
    __shared__ double red[kNRed][16];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
    for (int k = 0; k < kNRed; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) red[k][wave] = s;
    }
    __syncthreads();
    if (tid < kNRed) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[tid][w];
        partial[(long long)tile * kNRed + tid] = s;
    }
}

template <class L, class C, bool SNAP>
__device__ __forceinline__ void check_values(const Moments<L, C> &m, bool valid, C *__restrict__ snap,
                                             long long node, long long nodes, double (&v)[kNRed])
{
#pragma unroll
    for (int k = 0; k < kNRed; ++k) v[k] = 0.0;
    if (!valid) return;
    bool finite = isfinite((double)m.P) && isfinite((double)m.trJ);
#pragma unroll
    for (int b = 0; b < L::D; ++b) {
        const double u = (double)m.u[b];
        v[1] += u * u;
        if (SNAP) {
            const double du = u - (double)snap[b * nodes + node];
            v[0] += du * du;
            snap[b * nodes + node] = m.u[b];
        }
    }
#pragma unroll
    for (int a = 0; a <= L::D; ++a) {
        v[2 + a] = (double)m.ubar[a];
        finite = finite && isfinite((double)m.ubar[a]);
    }
    v[6] = (double)m.trJ;
    v[7] = finite ? 0.0 : 1.0;
}

// ----------------------------------------------------------------- kernels

// One tile of one time step: pull, wall rule, moments, optional fields and
// check, collision + forcing, write.  Shared by the single-case and the
// batched kernels, so both produce bitwise identical populations.
template <class L, int ST, bool EMIT, bool CHECK, bool MASK, bool NTST = false, bool WIDE = true>
__device__ __forceinline__ void step_tile(const KCase &p, int gx, int gy, int tile,
                                          const typename Store<ST>::T *__restrict__ src,
                                          typename Store<ST>::T *__restrict__ dst, const uint8_t *__restrict__ links,
                                          uint32_t fields, typename Store<ST>::C *__restrict__ out,
                                          typename Store<ST>::C *__restrict__ snap, double *__restrict__ partial)
{
    using S = Store<ST>;
    using C = typename S::C;
    const int tx = tile % gx, rest = tile / gx;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = (rest % gy) * blockDim.y + threadIdx.y;
    const int z = rest / gy;
    const bool inside = (x < p.nx) && (y < p.ny);
    Node<L, C> n;
    Moments<L, C> m;
    bool fluid = false;
    __builtin_amdgcn_s_setprio(2);          // issue the node's loads ahead of other waves' arithmetic
    if (inside) fluid = gather<L, ST, MASK, true, WIDE>(p, src, links, x, y, z, n);
    __builtin_amdgcn_s_setprio(0);
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    const long long node = ((long long)z * p.ny + y) * p.nx + x;
    if (fluid) {
        moments<L, C>(p, n, m);
        if (EMIT) write_fields<L, C>(p, n, m, fields, out, grid_ix<WIDE>(x, y, z, p.ny, p.nx), nodes);
        const auto own = grid_ix<WIDE>(x, y, z, p.ny, p.pitch);
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            C fo[L::Q];
            collide_fused<L, C>(p, n, m, a, fo, m.fb[a + L::A0]);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                if (i >= qset<L>(a + L::A0)) continue;
                S::template store_hint<NTST>(dst + plane_of<L>(a, i) * p.dstride, own, fo[i],
                                             rest_value<L, C>(p, a, i), p.inv_scale);
            }
        }
    } else if (EMIT && inside) {
        // solid node: every emitted channel is zero
        write_zero_fields<L, C>(fields, out, node, nodes);
    }
    if (CHECK) {
        double v[kNRed];
        check_values<L, C, true>(m, fluid, snap, node, nodes, v);
        block_reduce_store(v, partial, tile);
    }
}

// Vector form of step_tile(): thread (tx, ty) of a tile owns the VX nodes
// x0 = (tile_x * bx + tx) * VX .. x0 + VX - 1 of its row; the tile covers
// bx * VX by by nodes.  Per node the arithmetic is exactly step_tile()'s, so
// populations and fields are bitwise those of the scalar kernel.
template <class L, int ST, bool EMIT, bool CHECK, bool MASK, int VX>
__device__ __forceinline__ void step_tile_vec(const KCase &p, int gx, int gy, int tile,
                                              const typename Store<ST>::T *__restrict__ src,
                                              typename Store<ST>::T *__restrict__ dst,
                                              const uint8_t *__restrict__ links, uint32_t fields,
                                              typename Store<ST>::C *__restrict__ out,
                                              typename Store<ST>::C *__restrict__ snap, double *__restrict__ partial)
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    const int tx = tile % gx, rest = tile / gx;
    const int x0 = (tx * blockDim.x + threadIdx.x) * VX;
    const int y = (rest % gy) * blockDim.y + threadIdx.y;
    const int z = rest / gy;
    const bool rowok = (x0 < p.nx) && (y < p.ny);
    const int lane = (threadIdx.y * blockDim.x + threadIdx.x) & 63;
    const bool fix_lo = (threadIdx.x == 0) || (lane == 0);
    const bool fix_hi = (threadIdx.x == blockDim.x - 1) || (lane == 63);
    Node<L, C> n[VX];
    bool fluid[VX];
    gather_vec<L, ST, MASK, VX>(p, src, links, x0, y, z, rowok, fix_lo, fix_hi, n, fluid);
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    const long long own = ((long long)z * p.ny + y) * p.pitch + x0;
    bool all_fluid = true;
#pragma unroll
    for (int v = 0; v < VX; ++v) all_fluid = all_fluid && fluid[v];
    double acc[kNRed];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) acc[k] = 0.0;
    Moments<L, C> m[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const long long node = ((long long)z * p.ny + y) * p.nx + x0 + v;
        const bool inside = rowok && (x0 + v < p.nx);
        if (fluid[v]) {
            moments<L, C>(p, n[v], m[v]);
            if (EMIT) write_fields<L, C>(p, n[v], m[v], fields, out, node, nodes);
        } else if (EMIT && inside) {
            write_zero_fields<L, C>(fields, out, node, nodes);
        }
        if (CHECK) {
            double vv[kNRed];
            check_values<L, C, true>(m[v], fluid[v], snap, node, nodes, vv);
#pragma unroll
            for (int k = 0; k < kNRed; ++k) acc[k] += vv[k];
        }
    }
#pragma unroll
    for (int a = 0; a < L::NS; ++a) {
        // collide set a of every owned node in place, then store plane by plane
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            if (!fluid[v]) continue;
            C fo[L::Q];
            collide_fused<L, C>(p, n[v], m[v], a, fo, m[v].fb[a + L::A0]);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) n[v].f[a][i] = fo[i];
        }
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (i >= qset<L>(a + L::A0)) continue;
            T *plane = dst + plane_of<L>(a, i) * p.dstride;
            const C rest_i = rest_value<L, C>(p, a, i);
            VecT<T, VX> ov;
#pragma unroll
            for (int v = 0; v < VX; ++v) ov.v[v] = fluid[v] ? S::encode(n[v].f[a][i], rest_i, p.inv_scale) : T(0);
            if (all_fluid) {
                vstore<T, VX>(plane + own, ov);
            } else {
#pragma unroll
                for (int v = 0; v < VX; ++v)
                    if (fluid[v]) plane[own + v] = ov.v[v];
            }
        }
    }
    if (CHECK) block_reduce_store(acc, partial, tile);
}

template <class L, int ST, bool EMIT, bool CHECK, bool MASK, int VX, bool NTST = false, bool WIDE = true>
__global__ void __launch_bounds__(256)
k_step(KCase p, Tiling tl, const typename Store<ST>::T *__restrict__ src, typename Store<ST>::T *__restrict__ dst,
       const uint8_t *__restrict__ links, uint32_t fields, typename Store<ST>::C *__restrict__ out,
       typename Store<ST>::C *__restrict__ snap, double *__restrict__ partial)
{
    if constexpr (VX == 1)
        step_tile<L, ST, EMIT, CHECK, MASK, NTST, WIDE>(p, tl.gx, tl.gy, block_tile(tl), src, dst, links, fields,
                                                      out, snap, partial);
    else
        step_tile_vec<L, ST, EMIT, CHECK, MASK, VX>(p, tl.gx, tl.gy, block_tile(tl), src, dst, links, fields, out,
                                                    snap, partial);
}

// ----------------------------------------------------------------- two steps per pass (2D, axis links)

// Output rows of one tile of k_step2 per storage.  The LDS copy of the
// intermediate state (NS * Q planes of (64 + 2) x (rows + 2) stored values)
// is 47.5 KB for FP64, 39.6 KB for FP32 and 19.8 KB for the 16-bit formats
// (D2Q5, three sets).  The 16-bit formats keep 8 rows rather than 16: their
// step 1 then pulls the halo tile in one batch of three nodes per thread,
// not two, and more blocks fit per CU (measured +19-25 % at 4096^2 and
// 8192^2).
template <int ST> struct Fuse2Rows { static constexpr int TY = 8, NT = 256; };
template <> struct Fuse2Rows<MDF_F64> { static constexpr int TY = 4, NT = 256; };

constexpr int kF2X = 64;                 // output columns of a tile
constexpr int kF2W = kF2X + 2;           // columns of the tile plus its one-node halo
constexpr int kF2Strip = 16;             // tiles per strip of the two-step tile walk

// Two-step tile t of a gx x gy grid, walked in vertical strips kF2Strip
// tiles wide (the last strip takes the remaining columns): the tiles of one
// strip row are consecutive and the strip's rows follow each other, so a
// tile's neighbours in y run shortly before and after it, in the same XCD
// band, while the halo rows they share are still in that XCD's L2.  Row by
// row over a wide grid, one row of tiles (8192 x 10 rows x 15 FP32 planes,
// 4.9 MB) would exceed the L2 before the next row reused its halo.  A
// bijection on [0, gx * gy); with gx <= kF2Strip it is the row-major order.
__device__ __forceinline__ void strip_tile(int t, int gx, int gy, int &tx, int &ty)
{
    const int full = gx / kF2Strip;        // strips of full width
    const int per = kF2Strip * gy;         // tiles in one full strip
    const int s = t / per;
    if (s < full) {
        const int r = t - s * per;
        ty = r / kF2Strip;
        tx = s * kF2Strip + r % kF2Strip;
    } else {
        const int w = gx - full * kF2Strip;
        const int r = t - full * per;
        ty = r / w;
        tx = full * kF2Strip + r % w;
    }
}

// Two time steps in one pass over HBM (temporal blocking, 2D).  A block
// owns a tile of 64 x TY nodes.  Step 1 runs on the tile and a one-node
// halo with the one-step code (pull from the post-collision state f*(t) in
// HBM, wall rule, moments, collision); its result f*(t+1) goes to LDS in the
// storage format (encoded exactly as a one-step launch would store it).
// Halo nodes across a periodic face are the wrapped nodes; halo nodes behind
// a wall are not needed (step 2 takes the wall rule there).  Step 2 pulls
// f(t+2) from LDS, applies the same wall rule, emits the fields and writes
// f*(t+2) to HBM.  The fields of step 1 are not written: the emission buffer
// holds the fields of the latest step, and step 2 overwrites the same
// channels.  Every population, field and emitted value is bitwise that of
// two one-step launches; HBM traffic per step drops from one read and one
// write of the state to about half of that plus the halo re-reads
// ((64 + 2)(TY + 2) / (64 TY) of a read per two steps).
// The caller keeps f*(t+1) out of HBM, so the buffer the read kernels pull
// from is stale after this kernel until the next one-step launch.
template <class L, int ST>
struct Step2Lds {
    static constexpr int NE = kF2W * (Fuse2Rows<ST>::TY + 2);
    typename Store<ST>::T v[L::NS * L::Q * NE];
};

template <class L, int ST, bool EMIT, bool MASK, bool NTST = false, bool WIDE = true>
__device__ __forceinline__ void step2_tile(const KCase &p, int gx, int gy, int tile, const typename Store<ST>::T *__restrict__ src,
                                           typename Store<ST>::T *__restrict__ dst, const uint8_t *__restrict__ links,
                                           uint32_t fields, typename Store<ST>::C *__restrict__ out,
                                           typename Store<ST>::T *__restrict__ lds)
{
    static_assert(L::D == 2, "two-step tiles are two-dimensional");
    using S = Store<ST>;
    using C = typename S::C;
    constexpr int TY = Fuse2Rows<ST>::TY, NT = Fuse2Rows<ST>::NT;
    constexpr int W = kF2W, NE = kF2W * (TY + 2);
    int tx, ty;
    strip_tile(tile, gx, gy, tx, ty);
    const int x0 = tx * kF2X, y0 = ty * TY;
    const int tid = threadIdx.x;
    const long long nodes = (long long)p.nx * p.ny;

    // step 1: t -> t+1 on the tile and its halo, into LDS.  A thread owns
    // the halo-tile nodes tid, tid + 256, ...; G of them are pulled before
    // any is computed, so that (FP32, FP64) G nodes' loads are in flight
    // together (occupancy is bounded by LDS, not by registers).  The 16-bit
    // formats decode each node's values before the next node's loads.
    constexpr int K1 = (NE + NT - 1) / NT;
    constexpr int G = K1 < 3 ? K1 : 3;
#pragma unroll
    for (int k0 = 0; k0 < K1; k0 += G) {
        Node<L, C> n[G];
        bool fluid[G];
        // issue this batch's loads ahead of other waves' arithmetic
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int e = tid + (k0 + g) * NT;
            fluid[g] = false;
            if (k0 + g >= K1 || e >= NE) continue;
            const int ex = e % W, ey = e / W;
            int x = x0 - 1 + ex, y = y0 - 1 + ey;
            if (x < 0 || x >= p.nx) {
                if (p.bc[x < 0 ? 0 : 1] == MDF_WALL) continue;
                x = ((x % p.nx) + p.nx) % p.nx;
            }
            if (y < 0 || y >= p.ny) {
                if (p.bc[y < 0 ? 2 : 3] == MDF_WALL) continue;
                y = ((y % p.ny) + p.ny) % p.ny;
            }
            fluid[g] = gather<L, ST, MASK, true, WIDE>(p, src, links, x, y, 0, n[g]);   // false: solid node
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (!fluid[g]) continue;
            const int e = tid + (k0 + g) * NT;
            Moments<L, C> m;
            moments<L, C>(p, n[g], m);
            if (EMIT && (fields & MDF_FIELD_ACCUMULATE)) {
                // accumulated fields count every step: step 1's fields of
                // the tile's own nodes (not of its halo)
                const int ex = e % W, ey = e / W;
                const int x = x0 - 1 + ex, y = y0 - 1 + ey;
                if (ex >= 1 && ex <= kF2X && ey >= 1 && ey <= TY && x < p.nx && y < p.ny)
                    write_fields<L, C>(p, n[g], m, fields, out, grid_ix<WIDE>(x, y, 0, p.ny, p.nx), nodes);
            }
#pragma unroll
            for (int a = 0; a < L::NS; ++a) {
                C fo[L::Q];
                collide_fused<L, C>(p, n[g], m, a, fo, m.fb[a + L::A0]);
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    lds[(a * L::Q + i) * NE + e] = S::encode(fo[i], rest_value<L, C>(p, a, i), p.inv_scale);
            }
        }
    }
    __syncthreads();

    // step 2: t+1 -> t+2 on the tile, from LDS to HBM
    for (int e = tid; e < kF2X * TY; e += NT) {
        const int ox = e % kF2X, oy = e / kF2X;
        const int x = x0 + ox, y = y0 + oy;
        if (x >= p.nx || y >= p.ny) continue;
        const auto own = grid_ix<WIDE>(x, y, 0, p.ny, p.pitch);
        const auto node = grid_ix<WIDE>(x, y, 0, p.ny, p.nx);
        const int le = (oy + 1) * W + (ox + 1);
        unsigned lb = 0;
        if (MASK) lb = *elem(links, own);
        if (MASK && (lb & 0x80u)) {
            if (EMIT) {
                write_zero_fields<L, C>(fields, out, node, nodes);
            }
            continue;
        }
        Node<L, C> n;
        load_sources<L, C>(p, (long long)y * p.nx + x, n);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            int sx, sy, sz;            // (upstream values come from the LDS tile)
            const int face = pull_face<L, MASK, true, WIDE>(p, links, lb, x, y, 0, i, sx, sy, sz);
            const C w = C(L::w[i]);
            if (face < 0) {
                const int k = le - L::cx[i] - L::cy[i] * W;
#pragma unroll
                for (int a = 0; a < L::NS; ++a)
                    n.f[a][i] = S::decode(lds[(a * L::Q + i) * NE + k], rest_value<L, C>(p, a, i), p.scale);
            } else {
                const int j = L::opp[i];
#pragma unroll
                for (int a = 0; a < L::NS; ++a) {
                    const C v = S::decode(lds[(a * L::Q + j) * NE + le], rest_value<L, C>(p, a, j), p.scale);
                    if (a + L::A0 == 0) {
                        n.f[a][i] = v;
                    } else {
                        const int b = a + L::A0 - 1;
                        const C uw = (face < 6) ? kpar<C>(p.wallu[face][b], p.walluf[face][b]) : C(0);
                        n.f[a][i] = -v + C(2) * w * uw;
                    }
                }
            }
        }
        Moments<L, C> m;
        moments<L, C>(p, n, m);
        if (EMIT) write_fields<L, C>(p, n, m, fields, out, node, nodes);
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            C fo[L::Q];
            collide_fused<L, C>(p, n, m, a, fo, m.fb[a + L::A0]);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                if (i >= qset<L>(a + L::A0)) continue;
                S::template store_hint<NTST>(dst + plane_of<L>(a, i) * p.dstride, own, fo[i],
                                             rest_value<L, C>(p, a, i), p.inv_scale);
            }
        }
    }
}

template <class L, int ST, bool EMIT, bool MASK, bool NTST = false, bool WIDE = true>
__global__ void __launch_bounds__(Fuse2Rows<ST>::NT)
k_step2(KCase p, Tiling tl, const typename Store<ST>::T *__restrict__ src, typename Store<ST>::T *__restrict__ dst,
        const uint8_t *__restrict__ links, uint32_t fields, typename Store<ST>::C *__restrict__ out)
{
    __shared__ Step2Lds<L, ST> lds;
    step2_tile<L, ST, EMIT, MASK, NTST, WIDE>(p, tl.gx, tl.gy, block_tile(tl), src, dst, links, fields, out, lds.v);
}

// Batched two steps per launch: the persistent walk of k_step_batch over
// the flat list of the active cases' two-step tiles (prefix offsets
// tile_start2, total meta[2]).
template <class L, int ST, bool EMIT, bool MASK, bool NTST = false, bool WIDE = true>
__global__ void __launch_bounds__(Fuse2Rows<ST>::NT)
k_step2_batch(const BatchEntry *__restrict__ tab, const int *__restrict__ meta,
              const int *__restrict__ tile_start2, const int *__restrict__ active, int parity, uint32_t fields,
              int groups)
{
    __shared__ Step2Lds<L, ST> lds;
    const int nact = meta[0], total = meta[2];
    const int G = gridDim.x;
    const int ng = (groups > 1 && G % groups == 0) ? groups : 1;
    const int g = blockIdx.x % ng, per = G / ng, slot = blockIdx.x / ng;
    const int band_lo = (int)((long long)total * g / ng), band_hi = (int)((long long)total * (g + 1) / ng);
    for (int t = band_lo + slot; t < band_hi; t += per) {
        int lo = 0, hi = nact - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_start2[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchEntry &e = tab[active[lo]];
        const int sel = (e.cur + parity) & 1;
        using T = typename Store<ST>::T;
        using C = typename Store<ST>::C;
        step2_tile<L, ST, EMIT, MASK, NTST, WIDE>(e.p, e.gx2, e.gy2, t - tile_start2[lo],
                                                  static_cast<const T *>(e.pop[sel]),
                                                  static_cast<T *>(e.pop[sel ^ 1]), e.links, fields,
                                                  static_cast<C *>(e.out), lds.v);
        __syncthreads();   // the next tile's step 1 overwrites the LDS this tile's step 2 reads
    }
}

// ----------------------------------------------------------------- two steps per pass (3D, axis links)

// Output tile of k_step2z per storage: TX x TY nodes of an x-y plane, one
// thread each, walking a chunk of z-planes.  A tile row is TX x (bytes per
// value) = 128 bytes (FP32, 16-bit) or 256 bytes (FP64): whole cache lines
// for every population plane.  The LDS copy of the intermediate state
// f*(t+1) (see Step2ZLds) is 68 KB for FP32, 70 KB for FP64 and 68 KB for
// the 16-bit formats' 64 x 8 tile (D3Q7, four sets), so two blocks fit a
// CU's 160 KB.
// MINW: waves per SIMD the kernel is compiled for (its register budget).
// The 16-bit formats take the 64 x 8 tile (a one-node ring of 28 % of the
// tile, against 53 % for 64 x 4) only with a budget of four waves per SIMD
// (128 VGPRs, some spilled), so that both 8-wave blocks fit a CU: at the
// 158 VGPRs the compiler would otherwise use, one does and the tile
// measured -13 %; with the budget it runs 3-4 % (FP16) and 2-5 % (BF16)
// faster than the 64 x 4 tile at the same budget, itself 5 % and 8 % faster
// than at the compiler's.  FP32 and FP64 are bound to two 4-wave blocks per
// CU by their LDS and keep the compiler's budget.
template <int ST> struct Fuse2Z { static constexpr int TX = 64, TY = 8, MINW = 4; };
template <> struct Fuse2Z<MDF_F32> { static constexpr int TX = 32, TY = 8, MINW = 1; };
template <> struct Fuse2Z<MDF_F64> { static constexpr int TX = 32, TY = 4, MINW = 1; };

// The directions of an axis-link 3D lattice by their z-component: the
// in-plane ones (c_z = 0) in lattice order, and the +z and -z links.
template <class L>
struct ZSplit {
    static constexpr int count_ip()
    {
        int n = 0;
        for (int i = 0; i < L::Q; ++i) n += (L::cz[i] == 0) ? 1 : 0;
        return n;
    }
    // rank of direction i among the in-plane directions (-1 for a z link)
    static constexpr int rank(int i)
    {
        if (L::cz[i] != 0) return -1;
        int r = 0;
        for (int k = 0; k < i; ++k) r += (L::cz[k] == 0) ? 1 : 0;
        return r;
    }
    static constexpr int find_z(int sgn)
    {
        for (int i = 0; i < L::Q; ++i)
            if (L::cz[i] == sgn) return i;
        return -1;
    }
    static constexpr int NIP = count_ip();
    static constexpr int ZP = find_z(1), ZM = find_z(-1);
};

// LDS of k_step2z: f*(t+1) of the planes step 2 reads, in the storage
// encoding.  Two in-plane slots (the plane step 2 works on and the next
// one) hold the in-plane directions of the TX x TY tile nodes and, of the
// halo ring (no corners), only the direction that streams into the tile:
// +x of the column left of the tile, -x right of it, +y below, -y above.
// Three z slots (planes z - 1, z, z + 1) hold the +z and -z directions of
// the tile nodes.
template <class L, int ST>
struct Step2ZLds {
    static constexpr int TX = Fuse2Z<ST>::TX, TY = Fuse2Z<ST>::TY;
    static constexpr int NI = TX * TY, NH = 2 * (TX + TY);
    static constexpr int IPS = L::NS * ZSplit<L>::NIP * NI + L::NS * NH;   // one in-plane slot
    static constexpr int ZS = L::NS * 2 * NI;                              // one z slot
    typename Store<ST>::T v[2 * IPS + 3 * ZS];
};

// Which values of a plane's f*(t+1) step 1 keeps: everything step 2 reads
// (the planes step 2 works on), or only the +z (-z) links of the tile nodes
// (the plane below (above) the chunk).
enum { kZKeepAll = 0, kZKeepUp = 1, kZKeepDown = 2 };

// Step 1 of k_step2z on local plane r (global z = z0 - 1 + r): the one-step
// update from f*(t) in HBM to f*(t+1), for the tile nodes and (KEEP ==
// kZKeepAll) the halo ring, written to LDS.  Nodes behind a wall face are
// skipped (step 2 takes the wall rule there); across a periodic face the
// wrapped node is computed.  Each thread takes positions tid and tid + NT
// and pulls both nodes before computing either (FP32 and FP64 issue both
// nodes' loads together; the 16-bit formats decode each node's values
// before the next node's loads).
template <class L, int ST, int KEEP, bool EMIT, bool MASK, bool WIDE>
__device__ __forceinline__ void step2z_plane1(const KCase &p, const typename Store<ST>::T *__restrict__ src,
                                              const uint8_t *__restrict__ links, uint32_t fields,
                                              typename Store<ST>::C *__restrict__ out, int x0, int y0, int z,
                                              typename Store<ST>::T *__restrict__ ip,
                                              typename Store<ST>::T *__restrict__ zs)
{
    using S = Store<ST>;
    using C = typename S::C;
    using LD = Step2ZLds<L, ST>;
    using Z = ZSplit<L>;
    constexpr int TX = LD::TX, TY = LD::TY, NI = LD::NI, NH = LD::NH, NT = NI;
    constexpr int NPOS = (KEEP == kZKeepAll) ? NI + NH : NI;
    constexpr int G = (NPOS + NT - 1) / NT;
    const int tid = threadIdx.x;
    if (z < 0 || z >= p.nz) {
        if (p.bc[z < 0 ? 4 : 5] == MDF_WALL) return;
        z = ((z % p.nz) + p.nz) % p.nz;
    }
    Node<L, C> n[G];
    bool fluid[G];
    int pos[G];
    __builtin_amdgcn_s_setprio(2);          // issue the loads ahead of other waves' arithmetic
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int e = tid + g * NT;
        pos[g] = e;
        fluid[g] = false;
        if (e >= NPOS) continue;
        int lx, ly;
        if (e < NI) {
            lx = e % TX;
            ly = e / TX;
        } else {
            const int h = e - NI;
            if (h < TY) { lx = -1; ly = h; }
            else if (h < 2 * TY) { lx = TX; ly = h - TY; }
            else if (h < 2 * TY + TX) { lx = h - 2 * TY; ly = -1; }
            else { lx = h - 2 * TY - TX; ly = TY; }
        }
        int x = x0 + lx, y = y0 + ly;
        if (x < 0 || x >= p.nx) {
            if (p.bc[x < 0 ? 0 : 1] == MDF_WALL) continue;
            x = ((x % p.nx) + p.nx) % p.nx;
        }
        if (y < 0 || y >= p.ny) {
            if (p.bc[y < 0 ? 2 : 3] == MDF_WALL) continue;
            y = ((y % p.ny) + p.ny) % p.ny;
        }
        fluid[g] = gather<L, ST, MASK, true, WIDE>(p, src, links, x, y, z, n[g]);   // false: solid node
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (!fluid[g]) continue;
        const int e = pos[g];
        Moments<L, C> m;
        moments<L, C>(p, n[g], m);
        if (EMIT && KEEP == kZKeepAll && e < NI && (fields & MDF_FIELD_ACCUMULATE)) {
            // accumulated fields count every step: step 1's fields of the
            // tile's own nodes on the chunk's planes
            const int x = x0 + e % TX, y = y0 + e / TX;
            if (x < p.nx && y < p.ny)
                write_fields<L, C>(p, n[g], m, fields, out, grid_ix<WIDE>(x, y, z, p.ny, p.nx),
                                   (long long)p.nx * p.ny * p.nz);
        }
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            C fo[L::Q];
            collide_fused<L, C>(p, n[g], m, a, fo, m.fb[a + L::A0]);
            if (e < NI) {
                if (KEEP == kZKeepAll) {
#pragma unroll
                    for (int i = 0; i < L::Q; ++i) {
                        if (L::cz[i] != 0) continue;
                        ip[(a * Z::NIP + Z::rank(i)) * NI + e] = S::encode(fo[i], rest_value<L, C>(p, a, i), p.inv_scale);
                    }
                }
                if (KEEP != kZKeepDown)
                    zs[(a * 2 + 0) * NI + e] = S::encode(fo[Z::ZP], rest_value<L, C>(p, a, Z::ZP), p.inv_scale);
                if (KEEP != kZKeepUp)
                    zs[(a * 2 + 1) * NI + e] = S::encode(fo[Z::ZM], rest_value<L, C>(p, a, Z::ZM), p.inv_scale);
            } else {
                // a halo node keeps the one link that streams into the tile
                const int h = e - NI;
                int dir = 0;
#pragma unroll
                for (int i = 0; i < L::Q; ++i) {
                    if (h < TY && L::cx[i] == 1) dir = i;
                    else if (h >= TY && h < 2 * TY && L::cx[i] == -1) dir = i;
                    else if (h >= 2 * TY && h < 2 * TY + TX && L::cy[i] == 1) dir = i;
                    else if (h >= 2 * TY + TX && L::cy[i] == -1) dir = i;
                }
                C v = fo[0];
#pragma unroll
                for (int i = 1; i < L::Q; ++i)
                    if (i == dir) v = fo[i];
                ip[L::NS * Z::NIP * NI + a * NH + h] = S::encode(v, rest_value<L, C>(p, a, dir), p.inv_scale);
            }
        }
    }
}

// Step 2 of k_step2z on local plane r (global z): pull f(t+2) from the LDS
// copy of f*(t+1) with the same wall and solid rules, emit the fields, write
// f*(t+2) to HBM.
template <class L, int ST, bool EMIT, bool MASK, bool NTST, bool WIDE>
__device__ __forceinline__ void step2z_plane2(const KCase &p, typename Store<ST>::T *__restrict__ dst,
                                              const uint8_t *__restrict__ links, uint32_t fields,
                                              typename Store<ST>::C *__restrict__ out, int x0, int y0, int z,
                                              const typename Store<ST>::T *__restrict__ ip,
                                              const typename Store<ST>::T *__restrict__ zdown,
                                              const typename Store<ST>::T *__restrict__ zown,
                                              const typename Store<ST>::T *__restrict__ zup)
{
    using S = Store<ST>;
    using C = typename S::C;
    using LD = Step2ZLds<L, ST>;
    using Z = ZSplit<L>;
    constexpr int TX = LD::TX, TY = LD::TY, NI = LD::NI, NH = LD::NH;
    const int e = threadIdx.x;
    const int lx = e % TX, ly = e / TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= p.nx || y >= p.ny) return;
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    const auto own = grid_ix<WIDE>(x, y, z, p.ny, p.pitch);
    const auto node = grid_ix<WIDE>(x, y, z, p.ny, p.nx);
    unsigned lb = 0;
    if (MASK) lb = *elem(links, own);
    if (MASK && (lb & 0x80u)) {
        if (EMIT) {
            write_zero_fields<L, C>(fields, out, node, nodes);
        }
        return;
    }
    // LDS index of the stored value of direction j at the own node
    auto own_value = [&](int a, int j) -> C {
        typename S::T raw;
        if (L::cz[j] == 0) raw = ip[(a * Z::NIP + Z::rank(j)) * NI + e];
        else raw = zown[(a * 2 + (L::cz[j] > 0 ? 0 : 1)) * NI + e];
        return S::decode(raw, rest_value<L, C>(p, a, j), p.scale);
    };
    Node<L, C> n;
    load_sources<L, C>(p, ((long long)z * p.ny + y) * p.nx + x, n);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int sx, sy, sz;                // (upstream values come from the LDS slots)
        const int face = pull_face<L, MASK, true, WIDE>(p, links, lb, x, y, z, i, sx, sy, sz);
        const C w = C(L::w[i]);
        if (face < 0) {
#pragma unroll
            for (int a = 0; a < L::NS; ++a) {
                typename S::T raw;
                if (L::cz[i] > 0) {
                    raw = zdown[(a * 2 + 0) * NI + e];
                } else if (L::cz[i] < 0) {
                    raw = zup[(a * 2 + 1) * NI + e];
                } else {
                    const int ux = lx - L::cx[i], uy = ly - L::cy[i];
                    if (ux >= 0 && ux < TX && uy >= 0 && uy < TY) {
                        raw = ip[(a * Z::NIP + Z::rank(i)) * NI + uy * TX + ux];
                    } else {
                        int h;
                        if (ux < 0) h = uy;
                        else if (ux >= TX) h = TY + uy;
                        else if (uy < 0) h = 2 * TY + ux;
                        else h = 2 * TY + TX + ux;
                        raw = ip[L::NS * Z::NIP * NI + a * NH + h];
                    }
                }
                n.f[a][i] = S::decode(raw, rest_value<L, C>(p, a, i), p.scale);
            }
        } else {
            const int j = L::opp[i];
#pragma unroll
            for (int a = 0; a < L::NS; ++a) {
                const C v = own_value(a, j);
                if (a + L::A0 == 0) {
                    n.f[a][i] = v;
                } else {
                    const int b = a + L::A0 - 1;
                    const C uw = (face < 6) ? kpar<C>(p.wallu[face][b], p.walluf[face][b]) : C(0);
                    n.f[a][i] = -v + C(2) * w * uw;
                }
            }
        }
    }
    Moments<L, C> m;
    moments<L, C>(p, n, m);
    if (EMIT) write_fields<L, C>(p, n, m, fields, out, node, nodes);
#pragma unroll
    for (int a = 0; a < L::NS; ++a) {
        C fo[L::Q];
        collide_fused<L, C>(p, n, m, a, fo, m.fb[a + L::A0]);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (i >= qset<L>(a + L::A0)) continue;
            S::template store_hint<NTST>(dst + plane_of<L>(a, i) * p.dstride, own, fo[i],
                                         rest_value<L, C>(p, a, i), p.inv_scale);
        }
    }
}

// Two time steps in one pass over HBM on a 3D axis-link lattice (temporal
// blocking along z).  A block owns a TX x TY tile of an x-y plane and a chunk
// of zc planes z0 .. z1 - 1, and walks it plane by plane: step 1 advances
// the next plane (and a one-node halo ring in x and y) from f*(t) in HBM to
// f*(t+1) in LDS, then step 2 advances the current plane from the three
// planes of f*(t+1) around it to f*(t+2) in HBM.  The planes z0 - 1 and z1
// (across a periodic face: the wrapped planes) give step 2 their +z and -z
// links.  Every population, field and emitted value is bitwise that of two
// one-step launches; the state crosses HBM once per two steps, plus the
// halo ring ((TX + TY) 2 / (TX TY) of a read) and the two chunk-end planes
// (2 / zc of a read).  Like k_step2, f*(t+1) never reaches HBM.
template <class L, int ST, bool EMIT, bool MASK, bool NTST = false, bool WIDE = true>
__global__ void __launch_bounds__(Fuse2Z<ST>::TX * Fuse2Z<ST>::TY, Fuse2Z<ST>::MINW)
k_step2z(KCase p, Tiling tl, const typename Store<ST>::T *__restrict__ src, typename Store<ST>::T *__restrict__ dst,
         const uint8_t *__restrict__ links, uint32_t fields, typename Store<ST>::C *__restrict__ out)
{
    static_assert(L::D == 3 && !L::DIAG, "z-walking two-step tiles are for 3D axis-link lattices");
    using LD = Step2ZLds<L, ST>;
    using T = typename Store<ST>::T;
    __shared__ LD lds;
    const int tile = block_tile(tl);
    const int tx = tile % tl.gx, rest = tile / tl.gx;
    const int ty = rest % tl.gy, chunk = rest / tl.gy;
    const int x0 = tx * LD::TX, y0 = ty * LD::TY;
    const int z0 = chunk * tl.zc;
    const int z1 = (z0 + tl.zc < p.nz) ? z0 + tl.zc : p.nz;
    // local plane r is global plane z0 - 1 + r; its slots are in-plane slot
    // r % 2 and z slot r % 3
    T *const base = lds.v;
    auto ips = [&](int r) { return base + (r & 1) * LD::IPS; };
    auto zsl = [&](int r) { return base + 2 * LD::IPS + (r % 3) * LD::ZS; };
    step2z_plane1<L, ST, kZKeepUp, EMIT, MASK, WIDE>(p, src, links, fields, out, x0, y0, z0 - 1, ips(0), zsl(0));
    step2z_plane1<L, ST, kZKeepAll, EMIT, MASK, WIDE>(p, src, links, fields, out, x0, y0, z0, ips(1), zsl(1));
    const int nzc = z1 - z0;
    for (int r = 1; r <= nzc; ++r) {
        if (r < nzc)
            step2z_plane1<L, ST, kZKeepAll, EMIT, MASK, WIDE>(p, src, links, fields, out, x0, y0, z0 + r,
                                                              ips(r + 1), zsl(r + 1));
        else
            step2z_plane1<L, ST, kZKeepDown, EMIT, MASK, WIDE>(p, src, links, fields, out, x0, y0, z0 + r,
                                                               ips(r + 1), zsl(r + 1));
        __syncthreads();
        step2z_plane2<L, ST, EMIT, MASK, NTST, WIDE>(p, dst, links, fields, out, x0, y0, z0 + r - 1, ips(r),
                                                     zsl(r - 1), zsl(r), zsl(r + 1));
        __syncthreads();
    }
}

// Batched step: one persistent launch advances every active case of a
// context by one step.  The tiles of all active cases form one flat list
// (case k owns tiles tile_start[k] .. tile_start[k+1]-1); the grid is sized
// to the resident capacity of the chip and each block walks the list.  Tiles
// are dealt in XCD bands: blocks b with b % groups == g take the g-th
// contiguous band of the list, so neighbouring tiles of a case share an L2.
template <class L, int ST, bool EMIT, bool CHECK, bool MASK, int VX, bool NTST = false, bool WIDE = true>
__global__ void __launch_bounds__(256)
k_step_batch(const BatchEntry *__restrict__ tab, const int *__restrict__ meta, const int *__restrict__ tile_start,
             const int *__restrict__ active, int parity, uint32_t fields, int groups)
{
    const int nact = meta[0], total = meta[1];
    const int G = gridDim.x;
    const int ng = (groups > 1 && G % groups == 0) ? groups : 1;
    const int g = blockIdx.x % ng, per = G / ng, slot = blockIdx.x / ng;
    const int band_lo = (int)((long long)total * g / ng), band_hi = (int)((long long)total * (g + 1) / ng);
    for (int t = band_lo + slot; t < band_hi; t += per) {
        int lo = 0, hi = nact - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchEntry &e = tab[active[lo]];
        const int sel = (e.cur + parity) & 1;
        using T = typename Store<ST>::T;
        using C = typename Store<ST>::C;
        if constexpr (VX == 1)
            step_tile<L, ST, EMIT, CHECK, MASK, NTST, WIDE>(e.p, e.gx, e.gy, t - tile_start[lo],
                                                            static_cast<const T *>(e.pop[sel]),
                                                            static_cast<T *>(e.pop[sel ^ 1]), e.links, fields,
                                                            static_cast<C *>(e.out), static_cast<C *>(e.snap),
                                                            e.partial);
        else
            step_tile_vec<L, ST, EMIT, CHECK, MASK, VX>(e.p, e.gx, e.gy, t - tile_start[lo],
                                                        static_cast<const T *>(e.pop[sel]),
                                                        static_cast<T *>(e.pop[sel ^ 1]), e.links, fields,
                                                        static_cast<C *>(e.out), static_cast<C *>(e.snap), e.partial);
        if (CHECK) __syncthreads();   // the block reduction's LDS is reused by the next tile
    }
}

// Read-only pass at the current time: fields, populations or a check.
template <class L, int ST, bool MASK, bool PULL, int MODE>
__global__ void __launch_bounds__(256)
k_read(KCase p, Tiling tl, const typename Store<ST>::T *__restrict__ src, const uint8_t *__restrict__ links,
       uint32_t fields, typename Store<ST>::C *__restrict__ out, typename Store<ST>::C *__restrict__ snap,
       double *__restrict__ partial)
{
    using S = Store<ST>;
    using C = typename S::C;
    const int tile = block_tile(tl);
    const int tx = tile % tl.gx, rest = tile / tl.gx;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = (rest % tl.gy) * blockDim.y + threadIdx.y;
    const int z = rest / tl.gy;
    const bool inside = (x < p.nx) && (y < p.ny);
    Node<L, C> n;
    Moments<L, C> m;
    bool fluid = false;
    if (inside) fluid = gather<L, ST, MASK, PULL>(p, src, links, x, y, z, n);
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    const long long node = ((long long)z * p.ny + y) * p.nx + x;
    if (fluid) moments<L, C>(p, n, m);
    if (MODE == kReadFields && inside) {
        if (fluid) {
            write_fields<L, C>(p, n, m, fields, out, node, nodes);
        } else {
            write_zero_fields<L, C>(fields, out, node, nodes);
        }
    }
    if (MODE == kReadPops && inside) {
#pragma unroll
        for (int a = 0; a < L::NS; ++a)
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                out[(long long)(a * L::Q + i) * nodes + node] = fluid ? n.f[a][i] : C(0);
    }
    if (MODE == kReadCheck || MODE == kReadSums) {
        double v[kNRed];
        check_values<L, C, MODE == kReadCheck>(m, fluid, snap, node, nodes, v);
        block_reduce_store(v, partial, tile);
    }
}

// Initial state: f(x, 0) from fields (eq. 2-4, plus the inverse of eq. 3-16
// when a gradient is given) or from given populations.  Writes f(x, 0) into
// buffer `pre` (unshifted, read back locally at time 0) and the
// post-collision state f*(x, 0) into buffer `post`.
template <class L, int ST, bool MASK>
__global__ void __launch_bounds__(256)
k_init(KCase p, typename Store<ST>::T *__restrict__ pre, typename Store<ST>::T *__restrict__ post,
       const uint8_t *__restrict__ links, int kind, const typename Store<ST>::C *__restrict__ data)
{
    using S = Store<ST>;
    using C = typename S::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const long long own = ((long long)z * p.ny + y) * p.pitch + x;
    const long long nodes = (long long)p.nx * p.ny * p.nz;
    const long long node = ((long long)z * p.ny + y) * p.nx + x;
    if (MASK && (links[own] & 0x80u)) {
        for (int a = 0; a < L::NS; ++a)
            for (int i = 0; i < qset<L>(a + L::A0); ++i) {
                const long long k = plane_of<L>(a, i) * p.dstride + own;
                S::store(pre, k, rest_value<L, C>(p, a, i), rest_value<L, C>(p, a, i), p.inv_scale);
                S::store(post, k, rest_value<L, C>(p, a, i), rest_value<L, C>(p, a, i), p.inv_scale);
            }
        return;
    }
    Node<L, C> n;
    if (kind == MDF_INIT_POPULATIONS) {
#pragma unroll
        for (int a = 0; a < L::NS; ++a)
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                n.f[a][i] = i < qset<L>(a + L::A0) ? data[(long long)(a * L::Q + i) * nodes + node] : C(0);
    } else {
        C P = C(0), u[L::D];
#pragma unroll
        for (int b = 0; b < L::D; ++b) u[b] = C(0);
        if (kind != MDF_INIT_REST) {
            P = data[node];
#pragma unroll
            for (int b = 0; b < L::D; ++b) u[b] = data[(1 + b) * nodes + node];
        }
#pragma unroll
        for (int a = 0; a < L::NS; ++a) {
            const int pa = a + L::A0;
            const C ub = (pa == 0) ? C(p.rho0) : u[pa - 1];
            C flux[L::D], feq[L::Q];
#pragma unroll
            for (int b = 0; b < L::D; ++b) flux[b] = ub * u[b] + ((pa >= 1 && b == pa - 1) ? P : C(0));
            equilibrium<L, C>(ub, flux, feq, pa);
            if (L::R == 1) n.f[a][0] = feq[0];
#pragma unroll
            for (int i = L::R; i < L::Q; ++i) {
                if (i >= qset<L>(pa)) { n.f[a][i] = C(0); continue; }
                C cg = C(0);
#pragma unroll
                for (int b = 0; b < L::D; ++b) {
                    C g = C(0);
                    if (kind == MDF_INIT_FIELDS_GRAD && pa >= 1)
                        g = data[(1 + L::D + (pa - 1) * L::D + b) * nodes + node];
                    if (cdir<L>(i, b) > 0) cg += g;
                    else if (cdir<L>(i, b) < 0) cg -= g;
                }
                // f^eq (eq. 2-4) + f^ne with f^ne = -(1/s1) w_i c_i . grad u_a
                n.f[a][i] = feq[i] - (C(1) / C(p.s1)) * C(L::w[i]) * cg;
            }
            if (p.forcing == MDF_FORCING_SCHEME2) {
                // stored state fbar = f - w_i Fbar_a / 2, so that eq. 2-7a
                // gives back the initial ubar_a
                const C hf = C(0.5) * source_of<C>(p, pa, node);
                C moved = C(0);
#pragma unroll
                for (int i = L::R; i < L::Q; ++i) {
                    if (i == L::K || i >= qset<L>(pa)) continue;
                    const C whf = C(wset<L>(pa, i)) * hf;
                    n.f[a][i] -= whf;
                    moved += whf;
                }
                n.f[a][L::K] -= hf - moved;
            }
        }
    }
    load_sources<L, C>(p, node, n);
    Moments<L, C> m;
    moments<L, C>(p, n, m);
#pragma unroll
    for (int a = 0; a < L::NS; ++a) {
        C fo[L::Q];
        collide_fused<L, C>(p, n, m, a, fo, m.fb[a + L::A0]);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (i >= qset<L>(a + L::A0)) continue;
            const long long k = plane_of<L>(a, i) * p.dstride + own;
            S::store(pre, k, n.f[a][i], rest_value<L, C>(p, a, i), p.inv_scale);
            S::store(post, k, fo[i], rest_value<L, C>(p, a, i), p.inv_scale);
        }
    }
}

// Solid flags and upstream-solid link bits of every node (all zero when
// `solid` is null: a case without obstacles in a context where others have them).
template <class L>
__global__ void __launch_bounds__(256) k_links(KCase p, const uint8_t *__restrict__ solid, uint8_t *__restrict__ links)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const long long node = ((long long)z * p.ny + y) * p.nx + x;
    unsigned bits = (solid && solid[node]) ? 0x80u : 0u;
#pragma unroll
    for (int i = L::R; i < L::Q; ++i) {
        if (L::DIAG) break;               // diagonal lattices read the upstream flag instead
        int s[3] = {x - L::cx[i], y - L::cy[i], z - L::cz[i]};
        const int nn[3] = {p.nx, p.ny, p.nz};
        bool outside = false;
        for (int b = 0; b < 3; ++b) {
            if (s[b] < 0) { if (p.bc[2 * b] == MDF_WALL) outside = true; else s[b] += nn[b]; }
            else if (s[b] >= nn[b]) { if (p.bc[2 * b + 1] == MDF_WALL) outside = true; else s[b] -= nn[b]; }
        }
        if (!outside && solid && solid[((long long)s[2] * p.ny + s[1]) * p.nx + s[0]]) bits |= (1u << i);
    }
    links[((long long)z * p.ny + y) * p.pitch + x] = (uint8_t)bits;
}

// ----------------------------------------------------------------- dispatch

dim3 grid_of(const KCase &p, LaunchShape s)
{
    return dim3((p.nx + s.bx - 1) / s.bx, (p.ny + s.by - 1) / s.by, p.nz);
}

// Tiles of the step kernels (bx * vx by by nodes); the read kernels use
// one node per thread (vx = 1).
Tiling tiling_of(const KCase &p, LaunchShape s, int vx)
{
    Tiling t;
    t.gx = (p.nx + s.bx * vx - 1) / (s.bx * vx);
    t.gy = (p.ny + s.by - 1) / s.by;
    t.nb = t.gx * t.gy * p.nz;
    t.groups = s.groups > 1 ? s.groups : 1;
    return t;
}

template <class L, int ST>
hipError_t step_dispatch(const KCase &p, const CaseBufs &b, int src, bool check, uint32_t fields,
                         void *out, LaunchShape s, hipStream_t stream)
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    const T *in = static_cast<const T *>(b.pop[src]);
    T *o = static_cast<T *>(b.pop[src ^ 1]);
    C *emit = static_cast<C *>(out);
    C *snap = static_cast<C *>(b.snap);
    // the vector form exists for axis-link lattices only
    constexpr int VW = L::DIAG ? 1 : S::VX;
    const int vx = s.vx > 1 ? VW : 1;
    const Tiling tl = tiling_of(p, s, vx);
    const dim3 grid(tl.nb, 1, 1), block(s.bx, s.by, 1);
    const bool emit_on = (fields != 0) && out != nullptr;
    const bool mask = b.links != nullptr;
#define MDF_STEP_LAUNCH1(E, K, M, V, N, X)                                                                     \
    hipLaunchKernelGGL((k_step<L, ST, E, K, M, V, N, X>), grid, block, 0, stream, p, tl, in, o, b.links, fields, emit, \
                       snap, b.partial)
    // Working sets beyond the Infinity Cache: non-temporal stores and 32-bit
    // node offsets (measured +2 % there; -1 % on a 1024^2 grid inside the
    // cache, which keeps the 64-bit form).  Every plane and field channel
    // lies within 4 GiB: mdf_init refuses larger ones.
#define MDF_STEP_LAUNCH(E, K, M)                                                                   \
    do {                                                                                           \
        if (vx > 1) MDF_STEP_LAUNCH1(E, K, M, VW, false, true);                                    \
        else if (!p.ntstore) MDF_STEP_LAUNCH1(E, K, M, 1, false, true);                            \
        else MDF_STEP_LAUNCH1(E, K, M, 1, true, false);                                            \
    } while (0)
    if (mask) {
        if (emit_on) { if (check) MDF_STEP_LAUNCH(true, true, true); else MDF_STEP_LAUNCH(true, false, true); }
        else { if (check) MDF_STEP_LAUNCH(false, true, true); else MDF_STEP_LAUNCH(false, false, true); }
    } else {
        if (emit_on) { if (check) MDF_STEP_LAUNCH(true, true, false); else MDF_STEP_LAUNCH(true, false, false); }
        else { if (check) MDF_STEP_LAUNCH(false, true, false); else MDF_STEP_LAUNCH(false, false, false); }
    }
#undef MDF_STEP_LAUNCH
#undef MDF_STEP_LAUNCH1
    return hipGetLastError();
}

// z-planes per block of k_step2z: 32 where the grid gives enough blocks
// (the two chunk-end planes then cost 2/32 of a read), halved, down to 8,
// while a launch would have fewer than 512 blocks, the two per CU that every
// storage's LDS copy allows, so that small grids still fill the chip (at
// 128^3, chunks of 32 planes left 128 blocks of the 16-bit tile and 256 of
// the FP32 one).
inline int step2z_chunk(int nz, int tiles_xy)
{
    int zc = nz < 32 ? nz : 32;
    while (zc > 8 && (long long)tiles_xy * ((nz + zc - 1) / zc) < 512) zc /= 2;
    return zc;
}

template <class L, int ST>
hipError_t step2_dispatch(const KCase &p, const CaseBufs &b, int src, uint32_t fields, void *out, LaunchShape s,
                          hipStream_t stream)
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    if constexpr (L::DIAG) {
        return hipErrorInvalidValue;
    } else if constexpr (L::D == 3) {
        const T *in = static_cast<const T *>(b.pop[src]);
        T *o = static_cast<T *>(b.pop[src ^ 1]);
        C *emit = static_cast<C *>(out);
        constexpr int TX = Fuse2Z<ST>::TX, TY = Fuse2Z<ST>::TY;
        Tiling tl;
        tl.gx = (p.nx + TX - 1) / TX;
        tl.gy = (p.ny + TY - 1) / TY;
        tl.zc = step2z_chunk(p.nz, tl.gx * tl.gy);
        tl.nb = tl.gx * tl.gy * ((p.nz + tl.zc - 1) / tl.zc);
        tl.groups = s.groups > 1 ? s.groups : 1;
        const bool emit_on = (fields != 0) && out != nullptr;
        const bool mask = b.links != nullptr;
#define MDF_STEP2Z_LAUNCH1(E, M, N, X)                                                                   \
    hipLaunchKernelGGL((k_step2z<L, ST, E, M, N, X>), dim3(tl.nb), dim3(TX * TY), 0, stream, p, tl, in, o, \
                       b.links, fields, emit)
#define MDF_STEP2Z_LAUNCH(E, M)                                                                    \
    do {                                                                                           \
        if (!p.ntstore) MDF_STEP2Z_LAUNCH1(E, M, false, true);                                     \
        else MDF_STEP2Z_LAUNCH1(E, M, true, false);                                                \
    } while (0)
        if (mask) { if (emit_on) MDF_STEP2Z_LAUNCH(true, true); else MDF_STEP2Z_LAUNCH(false, true); }
        else { if (emit_on) MDF_STEP2Z_LAUNCH(true, false); else MDF_STEP2Z_LAUNCH(false, false); }
#undef MDF_STEP2Z_LAUNCH
#undef MDF_STEP2Z_LAUNCH1
        return hipGetLastError();
    } else {
        const T *in = static_cast<const T *>(b.pop[src]);
        T *o = static_cast<T *>(b.pop[src ^ 1]);
        C *emit = static_cast<C *>(out);
        Tiling tl;
        tl.gx = (p.nx + kF2X - 1) / kF2X;
        tl.gy = (p.ny + Fuse2Rows<ST>::TY - 1) / Fuse2Rows<ST>::TY;
        tl.nb = tl.gx * tl.gy;
        tl.groups = s.groups > 1 ? s.groups : 1;
        const bool emit_on = (fields != 0) && out != nullptr;
        const bool mask = b.links != nullptr;
#define MDF_STEP2_LAUNCH1(E, M, N, X)                                                                      \
    hipLaunchKernelGGL((k_step2<L, ST, E, M, N, X>), dim3(tl.nb), dim3(Fuse2Rows<ST>::NT), 0, stream, p, tl, in, o, \
                       b.links, fields, emit)
#define MDF_STEP2_LAUNCH(E, M)                                                                     \
    do {                                                                                           \
        if (!p.ntstore) MDF_STEP2_LAUNCH1(E, M, false, true);                                      \
        else MDF_STEP2_LAUNCH1(E, M, true, false);                                                 \
    } while (0)
        if (mask) { if (emit_on) MDF_STEP2_LAUNCH(true, true); else MDF_STEP2_LAUNCH(false, true); }
        else { if (emit_on) MDF_STEP2_LAUNCH(true, false); else MDF_STEP2_LAUNCH(false, false); }
#undef MDF_STEP2_LAUNCH
#undef MDF_STEP2_LAUNCH1
        return hipGetLastError();
    }
}

template <class L, int ST>
hipError_t read_dispatch(const KCase &p, const CaseBufs &b, int src, bool pull, int mode, uint32_t fields,
                         void *out, LaunchShape s, hipStream_t stream)
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    const T *in = static_cast<const T *>(b.pop[src]);
    C *o = static_cast<C *>(out);
    C *snap = static_cast<C *>(b.snap);
    const Tiling tl = tiling_of(p, s, 1);
    const dim3 grid(tl.nb, 1, 1), block(s.bx, s.by, 1);
    const bool mask = b.links != nullptr;
#define MDF_READ_LAUNCH(M, PL, MD) \
    hipLaunchKernelGGL((k_read<L, ST, M, PL, MD>), grid, block, 0, stream, p, tl, in, b.links, fields, o, snap, b.partial)
#define MDF_READ_MODE(M, PL)                                              \
    do {                                                                  \
        if (mode == kReadFields) MDF_READ_LAUNCH(M, PL, kReadFields);     \
        else if (mode == kReadPops) MDF_READ_LAUNCH(M, PL, kReadPops);    \
        else if (mode == kReadCheck) MDF_READ_LAUNCH(M, PL, kReadCheck);  \
        else MDF_READ_LAUNCH(M, PL, kReadSums);                           \
    } while (0)
    if (mask) { if (pull) MDF_READ_MODE(true, true); else MDF_READ_MODE(true, false); }
    else { if (pull) MDF_READ_MODE(false, true); else MDF_READ_MODE(false, false); }
#undef MDF_READ_MODE
#undef MDF_READ_LAUNCH
    return hipGetLastError();
}

template <class L, int ST>
hipError_t init_dispatch(const KCase &p, const CaseBufs &b, int cur, int kind, const void *data,
                         hipStream_t stream)
{
    using S = Store<ST>;
    using T = typename S::T;
    using C = typename S::C;
    T *post = static_cast<T *>(b.pop[cur]);
    T *pre = static_cast<T *>(b.pop[cur ^ 1]);
    const LaunchShape s{64, 4, 1};
    const dim3 grid = grid_of(p, s), block(s.bx, s.by, 1);
    if (b.links)
        hipLaunchKernelGGL((k_init<L, ST, true>), grid, block, 0, stream, p, pre, post, b.links, kind,
                           static_cast<const C *>(data));
    else
        hipLaunchKernelGGL((k_init<L, ST, false>), grid, block, 0, stream, p, pre, post, b.links, kind,
                           static_cast<const C *>(data));
    return hipGetLastError();
}

template <class L, int ST>
hipError_t batch_dispatch(const BatchLaunch &bl, bool check, bool emit, hipStream_t stream)
{
    using S = Store<ST>;
    constexpr int VW = L::DIAG ? 1 : S::VX;      // the vector form exists for axis-link lattices only
    const dim3 grid(bl.grid, 1, 1), block(bl.shape.bx, bl.shape.by, 1);
#define MDF_BATCH_LAUNCH1(E, K, M, V, N, X)                                                                  \
    hipLaunchKernelGGL((k_step_batch<L, ST, E, K, M, V, N, X>), grid, block, 0, stream, bl.tab, bl.meta,           \
                       bl.tile_start, bl.active, bl.parity, bl.fields, bl.shape.groups)
    // the store and offset forms of the single-case launches
#define MDF_BATCH_LAUNCH(E, K, M)                                                                  \
    do {                                                                                           \
        if (bl.shape.vx > 1) MDF_BATCH_LAUNCH1(E, K, M, VW, false, true);                          \
        else if (!bl.ntstore) MDF_BATCH_LAUNCH1(E, K, M, 1, false, true);                          \
        else MDF_BATCH_LAUNCH1(E, K, M, 1, true, false);                                           \
    } while (0)
    if (bl.mask) {
        if (emit) { if (check) MDF_BATCH_LAUNCH(true, true, true); else MDF_BATCH_LAUNCH(true, false, true); }
        else { if (check) MDF_BATCH_LAUNCH(false, true, true); else MDF_BATCH_LAUNCH(false, false, true); }
    } else {
        if (emit) { if (check) MDF_BATCH_LAUNCH(true, true, false); else MDF_BATCH_LAUNCH(true, false, false); }
        else { if (check) MDF_BATCH_LAUNCH(false, true, false); else MDF_BATCH_LAUNCH(false, false, false); }
    }
#undef MDF_BATCH_LAUNCH
#undef MDF_BATCH_LAUNCH1
    return hipGetLastError();
}

template <class L, int ST>
hipError_t batch2_dispatch(const BatchLaunch &bl, bool emit, hipStream_t stream)
{
    if constexpr (L::D != 2 || L::DIAG) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid(bl.grid, 1, 1), block(Fuse2Rows<ST>::NT, 1, 1);
#define MDF_BATCH2_LAUNCH1(E, M, N, X)                                                                    \
    hipLaunchKernelGGL((k_step2_batch<L, ST, E, M, N, X>), grid, block, 0, stream, bl.tab, bl.meta, bl.tile_start2, \
                       bl.active, bl.parity, bl.fields, bl.shape.groups)
#define MDF_BATCH2_LAUNCH(E, M)                                                                    \
    do {                                                                                           \
        if (!bl.ntstore) MDF_BATCH2_LAUNCH1(E, M, false, true);                                    \
        else MDF_BATCH2_LAUNCH1(E, M, true, false);                                                \
    } while (0)
        if (bl.mask) { if (emit) MDF_BATCH2_LAUNCH(true, true); else MDF_BATCH2_LAUNCH(false, true); }
        else { if (emit) MDF_BATCH2_LAUNCH(true, false); else MDF_BATCH2_LAUNCH(false, false); }
#undef MDF_BATCH2_LAUNCH
#undef MDF_BATCH2_LAUNCH1
        return hipGetLastError();
    }
}

template <class L, int ST>
hipError_t batch2_capacity(bool mask, int *blocks_per_cu)
{
    if constexpr (L::D != 2 || L::DIAG) {
        return hipErrorInvalidValue;
    } else {
        if (mask)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step2_batch<L, ST, true, true>,
                                                                Fuse2Rows<ST>::NT, 0);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step2_batch<L, ST, true, false>,
                                                            Fuse2Rows<ST>::NT, 0);
    }
}

template <class L, int ST>
hipError_t batch_capacity(LaunchShape shape, bool mask, int *blocks_per_cu)
{
    // resident blocks per CU of the heaviest variant (emit + check)
    using S = Store<ST>;
    constexpr int VW = L::DIAG ? 1 : S::VX;
    const int threads = shape.bx * shape.by;
    if (shape.vx > 1) {
        if (mask)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                blocks_per_cu, k_step_batch<L, ST, true, true, true, VW>, threads, 0);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                            k_step_batch<L, ST, true, true, false, VW>, threads, 0);
    }
    if (mask)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_batch<L, ST, true, true, true, 1>,
                                                            threads, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_batch<L, ST, true, true, false, 1>,
                                                        threads, 0);
}


#define MDF_DISPATCH_LAT(LAT, storage, FN, ...)                                              \
    switch (storage) {                                                                       \
    case MDF_F64: return FN<LAT, MDF_F64>(__VA_ARGS__);                                      \
    case MDF_F32: return FN<LAT, MDF_F32>(__VA_ARGS__);                                      \
    case MDF_F16DEV: return FN<LAT, MDF_F16DEV>(__VA_ARGS__);                                \
    case MDF_BF16DEV: return FN<LAT, MDF_BF16DEV>(__VA_ARGS__);                              \
    }


// Entry points of lattice L for every storage (the function-pointer table
// of LatOps); instantiating make_lat_ops<L> instantiates all of L's kernels.
template <class L>
hipError_t op_step(int storage, const KCase &p, const CaseBufs &b, int src, bool check, uint32_t fields,
                   void *out, LaunchShape s, hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, step_dispatch, p, b, src, check, fields, out, s, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_step2(int storage, const KCase &p, const CaseBufs &b, int src, uint32_t fields, void *out,
                    LaunchShape s, hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, step2_dispatch, p, b, src, fields, out, s, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_read(int storage, const KCase &p, const CaseBufs &b, int src, bool pull, int mode, uint32_t fields,
                   void *out, LaunchShape s, hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, read_dispatch, p, b, src, pull, mode, fields, out, s, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_init(int storage, const KCase &p, const CaseBufs &b, int cur, int kind, const void *data,
                   hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, init_dispatch, p, b, cur, kind, data, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_batch(int storage, const BatchLaunch &bl, bool check, bool emit, hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, batch_dispatch, bl, check, emit, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_batch2(int storage, const BatchLaunch &bl, bool emit, hipStream_t stream)
{
    MDF_DISPATCH_LAT(L, storage, batch2_dispatch, bl, emit, stream)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_batch_cap(int storage, LaunchShape shape, bool mask, int *blocks_per_cu)
{
    MDF_DISPATCH_LAT(L, storage, batch_capacity, shape, mask, blocks_per_cu)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_batch2_cap(int storage, bool mask, int *blocks_per_cu)
{
    MDF_DISPATCH_LAT(L, storage, batch2_capacity, mask, blocks_per_cu)
    return hipErrorInvalidValue;
}

template <class L>
hipError_t op_links(const KCase &p, const uint8_t *solid, uint8_t *links, hipStream_t stream)
{
    const LaunchShape s{64, 4, 1};
    const dim3 grid = grid_of(p, s), block(s.bx, s.by, 1);
    hipLaunchKernelGGL((k_links<L>), grid, block, 0, stream, p, solid, links);
    return hipGetLastError();
}

template <class L>
LatOps make_lat_ops()
{
    LatOps o;
    o.step = op_step<L>;
    o.step2 = op_step2<L>;
    o.read = op_read<L>;
    o.init = op_init<L>;
    o.batch = op_batch<L>;
    o.batch2 = op_batch2<L>;
    o.batch_cap = op_batch_cap<L>;
    o.batch2_cap = op_batch2_cap<L>;
    o.links = op_links<L>;
    o.cs2 = L::cs2;
    return o;
}

}  // namespace
}  // namespace mdf
