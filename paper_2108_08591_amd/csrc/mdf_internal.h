// mdf_internal.h -- declarations shared by the host API (mdf_api.cpp) and the
// HIP kernels (mdf_kernels.h and the lat_*.hip units).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "mdf.h"

namespace mdf {

// Number of FP64 reduction slots per check:
//   0: sum |u - u_snap|^2   1: sum |u|^2   2..5: sum ubar_a (a = 0..d)
//   6: sum_{a>=1} J_aa      7: count of nodes with a non-finite moment
constexpr int kNRed = 8;

// Per-case parameters as the kernels see them (passed by value).
struct KCase {
    int nx, ny, nz;
    int pitch;              // row stride of the population planes, elements
    long long dstride;      // elements from one (set, direction) plane to the next: nz*ny*pitch and a gap
    double s0, s1, s2;
    double rho0;
    double R;
    double fbar[4];         // Fbar_a, a = 0..d  (Fbar_0 = R, Fbar_a = F_a)
    double wallu[6][3];
    int bc[6];
    float scale, inv_scale; // 16-bit deviation storage: f = rest + scale * stored
    // the same parameters rounded to FP32 once on the host (the FP32 and
    // 16-bit kernels compute in FP32), and the rest populations w_i rho0 of
    // the set a = 0 (index 0: i = 0, index 1: i > 0)
    float s1f, s2f, rho0f, Rf;
    // cs^2 R / s1, the mass-source part of P (eq. 3-15), formed once on the
    // host in the operation order the kernels used to form it per node:
    // (cs^2 R) / s1, in FP64 and in FP32
    double rps;
    float rpsf;
    float fbarf[4];
    float walluf[6][3];
    double restd[3];        // w * rho0 by weight class: rest, axis, diagonal
    float restf[3];
    // optional per-node force, d x nodes values component-major in the
    // compute dtype (caller-owned device memory), added to fbar[1..d]
    const void *ffield;
    // forcing scheme: 0 = eq. 3-21, 1 = Scheme II (eq. 2-3c, 2-7a); fmove is
    // the factor of w_i Fbar on the moving populations (1, or 1 - s2/2)
    int forcing;
    double fmove;
    float fmovef;
    // 1: the step kernels write populations with a non-temporal hint (the
    // context's population buffers exceed the Infinity Cache)
    int ntstore;
};

// Device pointers of one case inside the workspace.
struct CaseBufs {
    void *pop[2];           // ping-pong population buffers (storage dtype)
    uint8_t *links;         // bit 7: solid node; bit i: upstream of direction i is solid
    void *snap;             // d * nodes velocity snapshot (compute dtype)
    double *partial;        // per-block reduction slots (kNRed each)
    double *result;         // kNRed reduced values
    int max_blocks;         // capacity of `partial`, in blocks
};

struct LaunchShape {
    int bx, by;             // threads per block along x and y (bx * by <= 256)
    int groups;             // > 1: hand out tiles in `groups` contiguous bands, one per XCD
    int vx;                 // > 1: step kernels give each thread the storage's vector width of x-nodes
    int fuse;               // 1: advance two steps per launch where possible (2D axis-link lattices)
};

// Tile grid of one launch: gx * gy * gz tiles of bx * by threads, launched
// as a 1D grid of nb = gx * gy * gz blocks.  zc: z-planes per tile of the
// three-dimensional two-step kernel (which walks a chunk of planes), else 1.
struct Tiling {
    int gx, gy, nb, groups;
    int zc = 1;
};

enum ReadMode { kReadFields = 0, kReadPops = 1, kReadCheck = 2, kReadSums = 3 };

// One case of a batched context, as the batched kernel reads it from device
// memory (the host keeps a mirror and uploads it before batched launches).
struct BatchEntry {
    KCase p;
    void *pop[2];
    const uint8_t *links;
    void *snap;
    double *partial;
    double *result;
    void *out;              // emitted fields of the current call, or null
    int gx, gy, ntiles;     // tile grid of the case for the batch launch shape
    int gx2, gy2, ntiles2;  // tile grid of two-step launches (2D axis-link lattices), else 0
    int cur;                // buffer holding f*(t) when the table was uploaded
};

// Arguments of one batched launch.
struct BatchLaunch {
    const BatchEntry *tab;  // device table (all cases)
    const int *meta;        // device: {active cases, total tiles}
    const int *tile_start;  // device: prefix offsets of the active cases' tiles
    const int *tile_start2; // device: the same for two-step tiles
    const int *active;      // device: case ids of the active cases
    int parity;             // launches since the table upload, mod 2
    uint32_t fields;        // emitted fields (0: none)
    int grid;               // blocks of the persistent launch
    bool mask;              // any case has obstacles
    bool ntstore;           // non-temporal stores and 32-bit node offsets
    LaunchShape shape;
};

// Entry points of one lattice for every storage.  Each lattice's kernels are
// instantiated in a translation unit of their own (lat_*.hip).
struct LatOps {
    hipError_t (*step)(int storage, const KCase &p, const CaseBufs &b, int src, bool check, uint32_t fields,
                       void *out, LaunchShape s, hipStream_t stream);
    hipError_t (*step2)(int storage, const KCase &p, const CaseBufs &b, int src, uint32_t fields, void *out,
                        LaunchShape s, hipStream_t stream);
    hipError_t (*read)(int storage, const KCase &p, const CaseBufs &b, int src, bool pull, int mode,
                       uint32_t fields, void *out, LaunchShape s, hipStream_t stream);
    hipError_t (*init)(int storage, const KCase &p, const CaseBufs &b, int cur, int kind, const void *data,
                       hipStream_t stream);
    hipError_t (*batch)(int storage, const BatchLaunch &bl, bool check, bool emit, hipStream_t stream);
    hipError_t (*batch2)(int storage, const BatchLaunch &bl, bool emit, hipStream_t stream);
    hipError_t (*batch_cap)(int storage, LaunchShape shape, bool mask, int *blocks_per_cu);
    hipError_t (*batch2_cap)(int storage, bool mask, int *blocks_per_cu);
    hipError_t (*links)(const KCase &p, const uint8_t *solid, uint8_t *links, hipStream_t stream);
    double cs2;             // the lattice's c_s^2 (of the velocity sets, on a lattice per set)
};
const LatOps &lat_ops_d2q5();
const LatOps &lat_ops_d3q7();
const LatOps &lat_ops_d2q5v();
const LatOps &lat_ops_d3q7v();
const LatOps &lat_ops_d2q4();
const LatOps &lat_ops_d3q6();
const LatOps &lat_ops_d2q4v();
const LatOps &lat_ops_d3q6v();
const LatOps &lat_ops_d2q9();
const LatOps &lat_ops_d3q15();
const LatOps &lat_ops_d2q9v();
const LatOps &lat_ops_d3q15v();
const LatOps &lat_ops_d2q9q5();
const LatOps &lat_ops_d3q15q7();

// Launchers (implemented in mdf_launch.hip).  All enqueue on `stream` and
// return the hipError_t of the launch.
hipError_t launch_links(int lattice, const KCase &p, const uint8_t *solid, uint8_t *links,
                        hipStream_t stream);
hipError_t launch_init(int lattice, int storage, const KCase &p, const CaseBufs &b, int cur,
                       int kind, const void *data, hipStream_t stream);
// Two steps in one launch (D2Q5, D2Q4 and their *_V forms): f*(t) in pop[src] -> f*(t+2) in
// pop[src ^ 1]; fields (if any) emitted at both steps.
hipError_t launch_step2(int lattice, int storage, const KCase &p, const CaseBufs &b, int src, uint32_t fields,
                        void *out, LaunchShape shape, hipStream_t stream);
hipError_t launch_step(int lattice, int storage, const KCase &p, const CaseBufs &b, int src,
                       bool check, uint32_t fields, void *out, LaunchShape shape,
                       int *nblocks_out, hipStream_t stream);
hipError_t launch_read(int lattice, int storage, const KCase &p, const CaseBufs &b, int src,
                       bool pull, int mode, uint32_t fields, void *out, LaunchShape shape,
                       int *nblocks_out, hipStream_t stream);
hipError_t launch_finalize(const CaseBufs &b, int nblocks, hipStream_t stream);
hipError_t launch_step_batch(int lattice, int storage, const BatchLaunch &bl, bool check, hipStream_t stream);
hipError_t batch_blocks_per_cu(int lattice, int storage, LaunchShape shape, bool mask, int *blocks_per_cu);
// Batched two steps per launch (the same lattices) over the two-step tile list.
hipError_t launch_step2_batch(int lattice, int storage, const BatchLaunch &bl, hipStream_t stream);
hipError_t batch2_blocks_per_cu(int lattice, int storage, bool mask, int *blocks_per_cu);
// Two-step tile grid of a case: tiles of 64 x rows nodes.
int step2_rows(int storage);
hipError_t launch_finalize_batch(const BatchEntry *tab, const int *meta, const int *active, int nactive,
                                 hipStream_t stream);

// Nodes per thread along x of the step kernels for a storage and shape.
int step_vx(int storage, LaunchShape shape);
// c_s^2 of a lattice's (velocity) sets, from its kernels' traits; 0 for an unknown id
double lattice_cs2(int lattice);
// Blocks of one step launch / one read launch.
int grid_blocks(const KCase &p, int storage, LaunchShape shape);
int read_blocks(const KCase &p, LaunchShape shape);

}  // namespace mdf
