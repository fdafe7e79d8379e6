// mdf_launch.hip -- lattice-independent launch helpers and reductions, and
// the routing of every launch to the entry points of its lattice (each
// lattice's kernels live in a translation unit of their own, lat_*.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdf_kernels.h"

namespace mdf {
namespace {

// Fixed-order sum of the per-block partials.
__global__ void __launch_bounds__(256) k_finalize(const double *__restrict__ partial, int nblocks, double *__restrict__ result)
{
    __shared__ double red[kNRed][256];
    const int t = threadIdx.x;
    double acc[kNRed];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) acc[k] = 0.0;
    for (int b = t; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < kNRed; ++k) acc[k] += partial[(long long)b * kNRed + k];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int k = 0; k < kNRed; ++k) red[k][t] += red[k][t + s];
        __syncthreads();
    }
    if (t < kNRed) result[t] = red[t][0];
}

// Fixed-order sum of each active case's per-tile partials (one block per case).
__global__ void __launch_bounds__(256)
k_finalize_batch(const BatchEntry *__restrict__ tab, const int *__restrict__ meta, const int *__restrict__ active)
{
    __shared__ double red[kNRed][256];
    if ((int)blockIdx.x >= meta[0]) return;
    const BatchEntry &e = tab[active[blockIdx.x]];
    const int t = threadIdx.x;
    double acc[kNRed];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) acc[k] = 0.0;
    for (int b = t; b < e.ntiles; b += 256)
#pragma unroll
        for (int k = 0; k < kNRed; ++k) acc[k] += e.partial[(long long)b * kNRed + k];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int k = 0; k < kNRed; ++k) red[k][t] += red[k][t + s];
        __syncthreads();
    }
    if (t < kNRed) e.result[t] = red[t][0];
}

const LatOps *ops_of(int lattice)
{
    switch (lattice) {
    case MDF_D2Q5: return &lat_ops_d2q5();
    case MDF_D3Q7: return &lat_ops_d3q7();
    case MDF_D2Q5_V: return &lat_ops_d2q5v();
    case MDF_D3Q7_V: return &lat_ops_d3q7v();
    case MDF_D2Q4: return &lat_ops_d2q4();
    case MDF_D3Q6: return &lat_ops_d3q6();
    case MDF_D2Q4_V: return &lat_ops_d2q4v();
    case MDF_D3Q6_V: return &lat_ops_d3q6v();
    case MDF_D2Q9: return &lat_ops_d2q9();
    case MDF_D3Q15: return &lat_ops_d3q15();
    case MDF_D2Q9_V: return &lat_ops_d2q9v();
    case MDF_D3Q15_V: return &lat_ops_d3q15v();
    case MDF_D2Q9_Q5: return &lat_ops_d2q9q5();
    case MDF_D3Q15_Q7: return &lat_ops_d3q15q7();
    }
    return nullptr;
}

bool two_d(int lattice)
{
    return lattice == MDF_D2Q5 || lattice == MDF_D2Q5_V || lattice == MDF_D2Q4 || lattice == MDF_D2Q4_V;
}

// lattices with axis links only (every lattice but D2Q9 / D3Q15 and their *_V forms)
bool axis_links(int lattice) { return lattice >= MDF_D2Q5 && lattice <= MDF_D3Q6_V; }

}  // namespace

double lattice_cs2(int lattice)
{
    const LatOps *o = ops_of(lattice);
    return o ? o->cs2 : 0.0;
}

int step_vx(int storage, LaunchShape s)
{
    if (s.vx <= 1) return 1;
    switch (storage) {
    case MDF_F64: return Store<MDF_F64>::VX;
    case MDF_F32: return Store<MDF_F32>::VX;
    case MDF_F16DEV: return Store<MDF_F16DEV>::VX;
    default: return Store<MDF_BF16DEV>::VX;
    }
}

int grid_blocks(const KCase &p, int storage, LaunchShape s)
{
    return tiling_of(p, s, step_vx(storage, s)).nb;
}

int read_blocks(const KCase &p, LaunchShape s)
{
    return tiling_of(p, s, 1).nb;
}

int step2_rows(int storage)
{
    switch (storage) {
    case MDF_F64: return Fuse2Rows<MDF_F64>::TY;
    case MDF_F32: return Fuse2Rows<MDF_F32>::TY;
    case MDF_F16DEV: return Fuse2Rows<MDF_F16DEV>::TY;
    default: return Fuse2Rows<MDF_BF16DEV>::TY;
    }
}

hipError_t launch_step(int lattice, int storage, const KCase &p, const CaseBufs &b, int src, bool check,
                       uint32_t fields, void *out, LaunchShape shape, int *nblocks_out, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    if (nblocks_out) *nblocks_out = grid_blocks(p, storage, shape);
    return o->step(storage, p, b, src, check, fields, out, shape, stream);
}

hipError_t launch_step2(int lattice, int storage, const KCase &p, const CaseBufs &b, int src, uint32_t fields,
                        void *out, LaunchShape shape, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o || !axis_links(lattice) || (two_d(lattice) && p.nz != 1)) return hipErrorInvalidValue;
    return o->step2(storage, p, b, src, fields, out, shape, stream);
}

hipError_t launch_read(int lattice, int storage, const KCase &p, const CaseBufs &b, int src, bool pull,
                       int mode, uint32_t fields, void *out, LaunchShape shape, int *nblocks_out,
                       hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    if (nblocks_out) *nblocks_out = read_blocks(p, shape);
    return o->read(storage, p, b, src, pull, mode, fields, out, shape, stream);
}

hipError_t launch_init(int lattice, int storage, const KCase &p, const CaseBufs &b, int cur, int kind,
                       const void *data, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    return o->init(storage, p, b, cur, kind, data, stream);
}

hipError_t launch_links(int lattice, const KCase &p, const uint8_t *solid, uint8_t *links, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    return o->links(p, solid, links, stream);
}

hipError_t launch_finalize(const CaseBufs &b, int nblocks, hipStream_t stream)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, stream, b.partial, nblocks, b.result);
    return hipGetLastError();
}

hipError_t launch_step2_batch(int lattice, int storage, const BatchLaunch &bl, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o || !two_d(lattice)) return hipErrorInvalidValue;
    return o->batch2(storage, bl, bl.fields != 0, stream);
}

hipError_t batch2_blocks_per_cu(int lattice, int storage, bool mask, int *blocks_per_cu)
{
    const LatOps *o = ops_of(lattice);
    if (!o || !two_d(lattice)) return hipErrorInvalidValue;
    return o->batch2_cap(storage, mask, blocks_per_cu);
}

hipError_t launch_step_batch(int lattice, int storage, const BatchLaunch &bl, bool check, hipStream_t stream)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    return o->batch(storage, bl, check, bl.fields != 0, stream);
}

hipError_t batch_blocks_per_cu(int lattice, int storage, LaunchShape shape, bool mask, int *blocks_per_cu)
{
    const LatOps *o = ops_of(lattice);
    if (!o) return hipErrorInvalidValue;
    return o->batch_cap(storage, shape, mask, blocks_per_cu);
}

hipError_t launch_finalize_batch(const BatchEntry *tab, const int *meta, const int *active, int nactive,
                                 hipStream_t stream)
{
    if (nactive <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_batch, dim3(nactive), dim3(256), 0, stream, tab, meta, active);
    return hipGetLastError();
}

}  // namespace mdf
