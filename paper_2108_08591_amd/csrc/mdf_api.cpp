// mdf_api.cpp -- host side of the C ABI declared in include/mdf.h.
//
// Owns only the host context: argument validation, the workspace layout
// (the caller's device memory), the ping-pong state of every case, kernel
// launches on the caller's stream and the FP64 residual / invariant
// read-back.  It never allocates device memory.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mdf.h"
#include "mdf_internal.h"

using mdf::CaseBufs;
using mdf::KCase;
using mdf::LaunchShape;

namespace {

thread_local std::string g_last_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Lattice ids: bit 0 selects 3D, bit 1 the velocity sets only (*_V), bit 2
// the lattices without a rest population (D2Q4, D3Q6), bit 3 those with
// diagonal links (D2Q9, D3Q15).  The two ids with a lattice per set
// (MDF_D2Q9_Q5, MDF_D3Q15_Q7: velocity sets with diagonal links, the set
// a = 0 on D2Q5 / D3Q7) are the exception to bit 2.
bool lat_mixed(int lattice) { return lattice == MDF_D2Q9_Q5 || lattice == MDF_D3Q15_Q7; }
bool lat_ok(int lattice) { return (lattice >= MDF_D2Q5 && lattice <= MDF_D3Q15_V) || lat_mixed(lattice); }
bool lat_2d(int lattice) { return (lattice & 1) == 0; }
bool lat_restfree(int lattice) { return (lattice & 4) != 0 && !lat_mixed(lattice); }
bool lat_diag(int lattice) { return (lattice & 8) != 0; }
// two steps per launch: lattices with axis links (2D tiles, or 3D tiles
// walking z-planes)
bool lat_fusable(int lattice) { return !lat_diag(lattice); }
// the default form: two steps per launch on the axis-link lattices, except
// 3D with 16-bit storage (measured slower there than one node per thread)
bool lat_fused_default(int lattice, int storage)
{
    if (lat_diag(lattice)) return false;
    if (lat_2d(lattice)) return true;
    return storage == MDF_F64 || storage == MDF_F32;
}
int lat_d(int lattice) { return lat_2d(lattice) ? 2 : 3; }
int lat_q(int lattice)
{
    if (lat_diag(lattice)) return lat_2d(lattice) ? 9 : 15;
    return lat_2d(lattice) ? (lat_restfree(lattice) ? 4 : 5) : (lat_restfree(lattice) ? 6 : 7);
}
// stored distribution sets: all d + 1, or the d velocity sets (the *_V lattices)
int lat_ns(int lattice) { return (lattice & 2) ? lat_d(lattice) : lat_d(lattice) + 1; }
// population planes of one buffer: every stored set has q directions, but for
// the set a = 0 of a lattice per set, which has 2d + 1
int lat_planes(int lattice)
{
    if (lat_mixed(lattice)) return 2 * lat_d(lattice) + 1 + lat_d(lattice) * lat_q(lattice);
    return lat_ns(lattice) * lat_q(lattice);
}
// weight of the rest (k = 0), axis (1) and diagonal (2) directions of the set
// a = 0 (eq. d2q5, d3q7, d2q4, d3q6, d2q9, d3q15; without a rest population
// the rest entry repeats the moving weight; a lattice per set takes the
// weights of D2Q5 / D3Q7 there)
double lat_wclass(int lattice, int k)
{
    if (lat_restfree(lattice)) return 1.0 / lat_q(lattice);
    if (lat_diag(lattice) && !lat_mixed(lattice)) {
        static const double w2[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0}, w3[3] = {2.0 / 9.0, 1.0 / 9.0, 1.0 / 72.0};
        return lat_2d(lattice) ? w2[k] : w3[k];
    }
    static const double w2[3] = {1.0 / 3.0, 1.0 / 6.0, 0.0}, w3[3] = {1.0 / 4.0, 1.0 / 8.0, 0.0};
    return lat_2d(lattice) ? w2[k] : w3[k];
}
size_t storage_bytes(int storage)
{
    switch (storage) {
    case MDF_F64: return 8;
    case MDF_F32: return 4;
    default: return 2;
    }
}
size_t compute_bytes(int storage) { return storage == MDF_F64 ? 8 : 4; }

// Row pitch: a whole number of 128-byte lines.
int row_pitch(int nx, int storage)
{
    const int per_line = int(128 / storage_bytes(storage));
    return (nx + per_line - 1) / per_line * per_line;
}

// Distance between consecutive population planes, in elements: the plane
// (nz * ny rows of the pitch) and a gap of 2304 bytes (nine 256-byte
// blocks).  On power-of-two grids the planes would otherwise all start a
// multiple of the plane size (32 MiB at 256^3 in FP16) apart, and the same
// offset of every plane, which the step kernels read at the same time, would
// fall in the same HBM channel and bank; shifted by 2304 bytes per plane, the
// one-step FP16 kernel ran 12 % faster at 256^3 and the 2D FP16 kernels
// 8-15 % faster at 4096^2-8192^2, with FP32 and FP64 within -2 % .. +6 %.
constexpr size_t kPlaneGapBytes = 2304;

size_t plane_stride(int nx, int ny, int nz, int storage)
{
    return size_t(row_pitch(nx, storage)) * ny * nz + kPlaneGapBytes / storage_bytes(storage);
}

struct CaseLayout {
    size_t pop[2], links, snap, partial, result;
    int max_blocks;
};

// Context-wide regions of the workspace (batched launches).
struct SharedLayout {
    size_t table, meta, tile_start, tile_start2, active;
};

// Blocks of the largest grid any allowed launch shape produces
// (bx >= 32, bx * by >= 64): at most ceil(nx/32) * ny * nz.
int max_blocks_of(const mdf_case &c) { return (c.nx + 31) / 32 * c.ny * c.nz; }

bool validate_case(int lattice, int storage, const mdf_case &c, std::string &why)
{
    char buf[256];
    const int d = lat_d(lattice);
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) { why = "grid sizes must be >= 1"; return false; }
    if (d == 2 && c.nz != 1) { why = "D2Q5 needs nz = 1"; return false; }
    const double nodes = double(c.nx) * c.ny * c.nz;
    if (nodes * lat_planes(lattice) > 2.0e9) { why = "case too large (>2e9 populations)"; return false; }
    // the step kernels address nodes by 32-bit byte offsets within a plane
    const double plane_bytes = double(row_pitch(c.nx, storage)) * c.ny * c.nz * storage_bytes(storage);
    if (plane_bytes > 4294967296.0 || nodes * compute_bytes(storage) > 4294967296.0) {
        why = "a population plane or field channel beyond 4 GiB";
        return false;
    }
    if (!(c.s1 > 0.0 && c.s1 < 2.0)) {
        snprintf(buf, sizeof buf, "s1 = %g outside (0, 2)", c.s1);
        why = buf;
        return false;
    }
    if (!(std::isfinite(c.s0) && c.s0 > 0.0 && c.s0 < 2.0)) { why = "s0 outside (0, 2)"; return false; }
    const double s2 = c.s2 > 0.0 ? c.s2 : 8.0 * (2.0 - c.s1) / (8.0 - c.s1);
    if (!(s2 > 0.0 && s2 < 2.0)) { why = "s2 outside (0, 2)"; return false; }
    if (!(c.rho0 > 0.0) || !std::isfinite(c.rho0)) { why = "rho0 must be > 0"; return false; }
    if (c.forcing != MDF_FORCING_PLAIN && c.forcing != MDF_FORCING_SCHEME2) {
        why = "forcing must be MDF_FORCING_PLAIN or MDF_FORCING_SCHEME2";
        return false;
    }
    for (int f = 0; f < 6; ++f) {
        if (c.bc[f] != MDF_PERIODIC && c.bc[f] != MDF_WALL) { why = "bc must be PERIODIC or WALL"; return false; }
        for (int b = 0; b < 3; ++b)
            if (!std::isfinite(c.wall_u[f][b])) { why = "non-finite wall velocity"; return false; }
    }
    for (int ax = 0; ax < 3; ++ax)
        if ((c.bc[2 * ax] == MDF_PERIODIC) != (c.bc[2 * ax + 1] == MDF_PERIODIC)) {
            why = "a periodic face must be paired with a periodic face";
            return false;
        }
    if (d == 2 && (c.bc[4] != MDF_PERIODIC || c.bc[5] != MDF_PERIODIC)) {
        why = "D2Q5 cases need periodic z faces";
        return false;
    }
    for (int b = 0; b < 3; ++b)
        if (!std::isfinite(c.force[b])) { why = "non-finite force"; return false; }
    if (!std::isfinite(c.R)) { why = "non-finite R"; return false; }
    return true;
}

size_t layout(int lattice, int storage, const mdf_case *cases, int ncases, bool has_solid,
              std::vector<CaseLayout> *out, SharedLayout *shared = nullptr)
{
    const int d = lat_d(lattice);
    size_t off = 0;
    if (out) out->resize(ncases);
    // per-case FP64 results, contiguous (one read-back for a whole batch)
    const size_t results = off;
    off = align256(off + size_t(ncases) * mdf::kNRed * sizeof(double));
    SharedLayout sh;
    sh.table = off;
    off = align256(off + size_t(ncases) * sizeof(mdf::BatchEntry));
    sh.meta = off;
    off = align256(off + 4 * sizeof(int));
    sh.tile_start = off;
    off = align256(off + size_t(ncases + 1) * sizeof(int));
    sh.tile_start2 = off;
    off = align256(off + size_t(ncases + 1) * sizeof(int));
    sh.active = off;
    off = align256(off + size_t(ncases) * sizeof(int));
    if (shared) *shared = sh;
    for (int k = 0; k < ncases; ++k) {
        const mdf_case &c = cases[k];
        CaseLayout L;
        const size_t plane = plane_stride(c.nx, c.ny, c.nz, storage);
        const size_t popb = size_t(lat_planes(lattice)) * plane * storage_bytes(storage);
        const size_t nodes = size_t(c.nx) * c.ny * c.nz;
        for (int b = 0; b < 2; ++b) { L.pop[b] = off; off = align256(off + popb); }
        L.links = off;
        if (has_solid) off = align256(off + plane);
        L.snap = off;
        off = align256(off + size_t(d) * nodes * compute_bytes(storage));
        L.max_blocks = max_blocks_of(c);
        L.partial = off;
        off = align256(off + size_t(L.max_blocks) * mdf::kNRed * sizeof(double));
        L.result = results + size_t(k) * mdf::kNRed * sizeof(double);
        if (out) (*out)[k] = L;
    }
    return off;
}

}  // namespace

struct GraphKey {
    int len, check, emit, parity, fuse;
    bool operator==(const GraphKey &o) const
    {
        return len == o.len && check == o.check && emit == o.emit && parity == o.parity && fuse == o.fuse;
    }
};

struct mdf_ctx {
    int lattice = 0, storage = 0, d = 2, q = 5, ncases = 0;
    std::vector<KCase> kc;
    std::vector<CaseBufs> bufs;
    std::vector<int> cur;              // buffer holding f*(., t)
    std::vector<int64_t> time;
    std::vector<int64_t> snap_time;    // time of the velocity snapshot, -1 = none
    std::vector<uint8_t> enabled;      // mdf_set_active
    LaunchShape shape{64, 4, 8, 1, 0};
    hipError_t latched = hipSuccess;
    std::string err;
    std::vector<double> host_red;
    // batched launches (ncases > 1)
    bool batched = false;
    bool any_mask = false;
    mdf::BatchEntry *d_tab = nullptr;
    int *d_meta = nullptr, *d_tile_start = nullptr, *d_tile_start2 = nullptr, *d_active = nullptr;
    double *d_results = nullptr;
    std::vector<mdf::BatchEntry> h_tab;
    std::vector<int> h_tile_start, h_tile_start2, h_active, h_meta;
    std::vector<double> h_results;
    int launches_since_upload = 0;       // buffer parity of the uploaded table
    int uploaded_fields = -1;
    int num_cu = 0;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    bool use_graphs = true;
    // graph bookkeeping reported by mdf_graph_stats
    int64_t graphs_captured = 0, graph_launches = 0, plain_chunks = 0, capture_failures = 0;
    std::string capture_error;
};

namespace {

mdf_status fail(mdf_ctx *ctx, mdf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_last_error = buf;
    return st;
}

mdf_status device_error(mdf_ctx *ctx, hipError_t e, const char *where)
{
    if (ctx) ctx->latched = e;
    return fail(ctx, MDF_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool case_ok(const mdf_ctx *ctx, int32_t case_id) { return case_id >= 0 && case_id < ctx->ncases; }

KCase make_kcase(int lattice, int storage, const mdf_case &c)
{
    KCase p;
    std::memset(&p, 0, sizeof p);
    p.nx = c.nx;
    p.ny = c.ny;
    p.nz = c.nz;
    p.pitch = row_pitch(c.nx, storage);
    p.dstride = (long long)plane_stride(c.nx, c.ny, c.nz, storage);
    p.s0 = c.s0;
    p.s1 = c.s1;
    p.s2 = c.s2 > 0.0 ? c.s2 : 8.0 * (2.0 - c.s1) / (8.0 - c.s1);
    p.rho0 = c.rho0;
    p.R = c.R;
    p.fbar[0] = c.R;
    for (int b = 0; b < lat_d(lattice); ++b) p.fbar[b + 1] = c.force[b];
    for (int f = 0; f < 6; ++f) {
        p.bc[f] = c.bc[f];
        for (int b = 0; b < 3; ++b) p.wallu[f][b] = c.wall_u[f][b];
    }
    const double scale = (storage == MDF_F16DEV || storage == MDF_BF16DEV) && c.u_ref > 0.0 ? c.u_ref : 1.0;
    p.scale = float(scale);
    p.inv_scale = float(1.0 / scale);
    p.s1f = float(p.s1);
    p.s2f = float(p.s2);
    p.rho0f = float(p.rho0);
    p.Rf = float(p.R);
    const double cs2 = mdf::lattice_cs2(lattice);
    p.rps = cs2 * p.R / p.s1;
    p.rpsf = float(cs2) * p.Rf / p.s1f;
    for (int a = 0; a < 4; ++a) p.fbarf[a] = float(p.fbar[a]);
    p.forcing = c.forcing;
    p.fmove = c.forcing == MDF_FORCING_SCHEME2 ? 1.0 - 0.5 * p.s2 : 1.0;
    p.fmovef = float(p.fmove);
    for (int f = 0; f < 6; ++f)
        for (int b = 0; b < 3; ++b) p.walluf[f][b] = float(p.wallu[f][b]);
    // rest weights of the lattice (eq. d2q5 / d3q7) times rho0
    for (int k = 0; k < 3; ++k) {
        p.restd[k] = lat_wclass(lattice, k) * p.rho0;
        p.restf[k] = float(p.restd[k]);
    }
    return p;
}

// Reduce the per-block partials of the last check/sums launch of case k and
// copy the kNRed results to the host.
mdf_status finalize_and_fetch(mdf_ctx *ctx, int k, int nblocks, hipStream_t st, double *out)
{
    hipError_t e = mdf::launch_finalize(ctx->bufs[k], nblocks, st);
    if (e != hipSuccess) return device_error(ctx, e, "finalize launch");
    e = hipMemcpyAsync(out, ctx->bufs[k].result, mdf::kNRed * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return device_error(ctx, e, "result copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error(ctx, e, "stream synchronize");
    return MDF_OK;
}

mdf_status step_case(mdf_ctx *ctx, int k, bool check, uint32_t fields, void *out, hipStream_t st,
                     int *nblocks)
{
    if (check && mdf::grid_blocks(ctx->kc[k], ctx->storage, ctx->shape) > ctx->bufs[k].max_blocks)
        return fail(ctx, MDF_EINVAL, "launch grid exceeds the reduction workspace");
    hipError_t e = mdf::launch_step(ctx->lattice, ctx->storage, ctx->kc[k], ctx->bufs[k], ctx->cur[k], check,
                                    fields, out, ctx->shape, nblocks, st);
    if (e != hipSuccess) return device_error(ctx, e, "step launch");
    ctx->cur[k] ^= 1;
    ctx->time[k] += 1;
    return MDF_OK;
}

// Advance case k by nsteps.  With the two-step form, pairs of steps run as
// one launch and the call always ends with at least one one-step launch, so
// that the buffer the read kernels pull from holds f*(t - 1) again; the
// check (if any) rides on the last step.
mdf_status advance_case(mdf_ctx *ctx, int k, int64_t nsteps, bool check_last, uint32_t fields, void *out,
                        hipStream_t st, int *nblocks)
{
    int64_t pairs = 0;
    if (ctx->shape.fuse && lat_fusable(ctx->lattice) && nsteps >= 3) pairs = (nsteps - 1) / 2;
    for (int64_t s = 0; s < pairs; ++s) {
        hipError_t e = mdf::launch_step2(ctx->lattice, ctx->storage, ctx->kc[k], ctx->bufs[k], ctx->cur[k], fields,
                                         out, ctx->shape, st);
        if (e != hipSuccess) return device_error(ctx, e, "two-step launch");
        ctx->cur[k] ^= 1;
        ctx->time[k] += 2;
    }
    const int64_t singles = nsteps - 2 * pairs;
    for (int64_t s = 0; s < singles; ++s) {
        mdf_status r = step_case(ctx, k, check_last && s == singles - 1, fields, out, st, nblocks);
        if (r != MDF_OK) return r;
    }
    return MDF_OK;
}

// Residual of case k from the reduced slots and the snapshot bookkeeping.
double residual_of(const mdf_ctx *ctx, int k, const double *red)
{
    const int64_t dt = ctx->time[k] - ctx->snap_time[k];
    if (ctx->snap_time[k] < 0 || dt <= 0) return INFINITY;
    const double den = std::sqrt(red[1]);
    if (!(den > 0.0)) return red[0] > 0.0 ? INFINITY : 0.0;
    return std::sqrt(red[0]) / (double(dt) * den);
}

// ---------------------------------------------------------------- batched path

void drop_graphs(mdf_ctx *ctx)
{
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
}

mdf_status batch_capacity_grid(mdf_ctx *ctx, int *grid)
{
    if (ctx->num_cu == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return device_error(ctx, e, "device query");
    }
    int per_cu = 0;
    hipError_t e = mdf::batch_blocks_per_cu(ctx->lattice, ctx->storage, ctx->shape, ctx->any_mask, &per_cu);
    if (e != hipSuccess) return device_error(ctx, e, "occupancy query");
    if (per_cu < 1) per_cu = 1;
    *grid = ctx->num_cu * per_cu;
    return MDF_OK;
}

// Fill the host mirror of the case table for the given active cases and
// emission targets, and copy it to the device.  Waits for the copies.
mdf_status batch_upload(mdf_ctx *ctx, const std::vector<int> &active, uint32_t fields, void *const *out,
                        hipStream_t st)
{
    const int n = ctx->ncases;
    ctx->h_tab.resize(n);
    for (int k = 0; k < n; ++k) {
        mdf::BatchEntry &e = ctx->h_tab[k];
        std::memset(&e, 0, sizeof e);
        e.p = ctx->kc[k];
        e.pop[0] = ctx->bufs[k].pop[0];
        e.pop[1] = ctx->bufs[k].pop[1];
        e.links = ctx->bufs[k].links;
        e.snap = ctx->bufs[k].snap;
        e.partial = ctx->bufs[k].partial;
        e.result = ctx->bufs[k].result;
        e.out = (fields && out) ? out[k] : nullptr;
        const int tile_x = ctx->shape.bx * mdf::step_vx(ctx->storage, ctx->shape);
        e.gx = (e.p.nx + tile_x - 1) / tile_x;
        e.gy = (e.p.ny + ctx->shape.by - 1) / ctx->shape.by;
        e.ntiles = e.gx * e.gy * e.p.nz;
        if (lat_2d(ctx->lattice)) {
            const int rows = mdf::step2_rows(ctx->storage);
            e.gx2 = (e.p.nx + 63) / 64;
            e.gy2 = (e.p.ny + rows - 1) / rows;
            e.ntiles2 = e.gx2 * e.gy2;
        }
        e.cur = ctx->cur[k];
        if (e.ntiles > ctx->bufs[k].max_blocks)
            return fail(ctx, MDF_EINVAL, "launch grid exceeds the reduction workspace");
    }
    ctx->h_active = active;
    ctx->h_tile_start.assign(active.size() + 1, 0);
    long long total = 0;
    for (size_t i = 0; i < active.size(); ++i) {
        ctx->h_tile_start[i] = int(total);
        total += ctx->h_tab[active[i]].ntiles;
    }
    if (total > 0x7fffffffLL) return fail(ctx, MDF_EINVAL, "batch has too many tiles");
    ctx->h_tile_start[active.size()] = int(total);
    ctx->h_tile_start2.assign(active.size() + 1, 0);
    long long total2 = 0;
    for (size_t i = 0; i < active.size(); ++i) {
        ctx->h_tile_start2[i] = int(total2);
        total2 += ctx->h_tab[active[i]].ntiles2;
    }
    if (total2 > 0x7fffffffLL) return fail(ctx, MDF_EINVAL, "batch has too many tiles");
    ctx->h_tile_start2[active.size()] = int(total2);
    ctx->h_meta = {int(active.size()), int(total), int(total2), 0};
    hipError_t e = hipMemcpyAsync(ctx->d_tab, ctx->h_tab.data(), sizeof(mdf::BatchEntry) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->d_meta, ctx->h_meta.data(), sizeof(int) * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !active.empty()) {
        e = hipMemcpyAsync(ctx->d_tile_start, ctx->h_tile_start.data(), sizeof(int) * (active.size() + 1),
                           hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->d_tile_start2, ctx->h_tile_start2.data(), sizeof(int) * (active.size() + 1),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->d_active, active.data(), sizeof(int) * active.size(), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error(ctx, e, "batch table upload");
    ctx->launches_since_upload = 0;
    ctx->uploaded_fields = int(fields);
    return MDF_OK;
}

mdf::BatchLaunch batch_args(mdf_ctx *ctx, uint32_t fields, int grid)
{
    mdf::BatchLaunch bl;
    bl.tab = ctx->d_tab;
    bl.meta = ctx->d_meta;
    bl.tile_start = ctx->d_tile_start;
    bl.tile_start2 = ctx->d_tile_start2;
    bl.active = ctx->d_active;
    bl.parity = 0;
    bl.fields = fields;
    bl.grid = grid;
    bl.mask = ctx->any_mask;
    bl.ntstore = ctx->kc[0].ntstore != 0;   // the same for every case of a context
    bl.shape = ctx->shape;
    return bl;
}

// nsteps batched steps of the uploaded active cases; the last one fused with
// the check when `check`.  With the two-step form (2D axis-link lattices), pairs of steps run
// as one launch of k_step2_batch and the chunk ends with at least one
// one-step launch (which carries the check and leaves f*(t - 1) in the other
// buffer for the read kernels).  A chunk whose length, form, check flag,
// emission and starting parity were seen before replays a captured graph.
mdf_status batch_steps(mdf_ctx *ctx, int nsteps, bool check, uint32_t fields, hipStream_t st)
{
    if (nsteps <= 0) return MDF_OK;
    int grid = 0;
    mdf_status r = batch_capacity_grid(ctx, &grid);
    if (r != MDF_OK) return r;
    const bool fuse = ctx->shape.fuse && lat_2d(ctx->lattice) && nsteps >= 3;
    const int pairs = fuse ? (nsteps - 1) / 2 : 0;
    const int singles = nsteps - 2 * pairs;
    int grid2 = 0;
    if (pairs > 0) {
        int per_cu = 0;
        hipError_t e = mdf::batch2_blocks_per_cu(ctx->lattice, ctx->storage, ctx->any_mask, &per_cu);
        if (e != hipSuccess) return device_error(ctx, e, "occupancy query");
        grid2 = ctx->num_cu * (per_cu < 1 ? 1 : per_cu);
    }
    mdf::BatchLaunch bl = batch_args(ctx, fields, grid);
    mdf::BatchLaunch bl2 = batch_args(ctx, fields, grid2);
    const int p0 = ctx->launches_since_upload & 1;
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        int launch = 0;
        for (int s = 0; s < pairs && e == hipSuccess; ++s, ++launch) {
            bl2.parity = (p0 + launch) & 1;
            e = mdf::launch_step2_batch(ctx->lattice, ctx->storage, bl2, st);
        }
        for (int s = 0; s < singles && e == hipSuccess; ++s, ++launch) {
            bl.parity = (p0 + launch) & 1;
            e = mdf::launch_step_batch(ctx->lattice, ctx->storage, bl, check && s == singles - 1, st);
        }
        return e;
    };
    const GraphKey key{nsteps, check ? 1 : 0, int(fields), p0, fuse ? 1 : 0};
    hipGraphExec_t exec = nullptr;
    for (auto &g : ctx->graphs)
        if (g.first == key) exec = g.second;
    if (!exec && ctx->use_graphs && st != nullptr && nsteps >= 4) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            e = enqueue();
            hipError_t e2 = hipStreamEndCapture(st, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e == hipSuccess) {
                ctx->graphs.push_back({key, exec});
                ctx->graphs_captured += 1;
            } else {
                exec = nullptr;
            }
            if (e != hipSuccess) {
                // capture unsupported on this stream: the context goes on with
                // plain launches, and mdf_graph_stats reports the failure
                ctx->capture_error = hipGetErrorString(e);
                (void)hipGetLastError();
                ctx->use_graphs = false;
                ctx->capture_failures += 1;
            }
        } else {
            ctx->capture_error = hipGetErrorString(e);
            (void)hipGetLastError();
            ctx->use_graphs = false;
            ctx->capture_failures += 1;
        }
    }
    if (exec) {
        hipError_t e = hipGraphLaunch(exec, st);
        if (e != hipSuccess) return device_error(ctx, e, "graph launch");
        ctx->graph_launches += 1;
    } else {
        hipError_t e = enqueue();
        if (e != hipSuccess) return device_error(ctx, e, "batched step launch");
        ctx->plain_chunks += 1;
    }
    const int launches = pairs + singles;
    ctx->launches_since_upload += launches;
    for (int k : ctx->h_active) {
        ctx->time[k] += nsteps;
        if (launches & 1) ctx->cur[k] ^= 1;
    }
    return MDF_OK;
}

// Reduce the fused check of the active cases and read every result back.
mdf_status batch_fetch_results(mdf_ctx *ctx, hipStream_t st)
{
    hipError_t e = mdf::launch_finalize_batch(ctx->d_tab, ctx->d_meta, ctx->d_active, int(ctx->h_active.size()), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_results.data(), ctx->d_results, sizeof(double) * ctx->h_results.size(),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error(ctx, e, "batch results");
    return MDF_OK;
}

}  // namespace

extern "C" {

size_t mdf_workspace_size(mdf_lattice lattice, mdf_storage storage, const mdf_case *cases, int32_t ncases,
                          int32_t has_solid)
{
    if (!lat_ok(lattice) || storage < MDF_F64 || storage > MDF_BF16DEV ||
        !cases || ncases < 1) {
        fail(nullptr, MDF_EINVAL, "mdf_workspace_size: invalid lattice, storage or cases");
        return 0;
    }
    std::string why;
    for (int k = 0; k < ncases; ++k)
        if (!validate_case(lattice, storage, cases[k], why)) {
            fail(nullptr, MDF_EINVAL, "mdf_workspace_size: case %d: %s", k, why.c_str());
            return 0;
        }
    return layout(lattice, storage, cases, ncases, has_solid != 0, nullptr);
}

mdf_status mdf_init(mdf_ctx **out, mdf_lattice lattice, mdf_storage storage, const mdf_case *cases,
                    int32_t ncases, void *workspace, size_t ws_bytes, const uint8_t *const *solid,
                    int32_t init_kind, const void *const *init_data, void *stream)
{
    if (!out) return fail(nullptr, MDF_EINVAL, "mdf_init: out is NULL");
    *out = nullptr;
    if (!lat_ok(lattice)) return fail(nullptr, MDF_EINVAL, "mdf_init: bad lattice");
    if (storage < MDF_F64 || storage > MDF_BF16DEV) return fail(nullptr, MDF_EINVAL, "mdf_init: bad storage");
    if (!cases || ncases < 1) return fail(nullptr, MDF_EINVAL, "mdf_init: no cases");
    if (init_kind < MDF_INIT_REST || init_kind > MDF_INIT_POPULATIONS)
        return fail(nullptr, MDF_EINVAL, "mdf_init: bad init_kind");
    if (!workspace) return fail(nullptr, MDF_EINVAL, "mdf_init: workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(nullptr, MDF_EINVAL, "mdf_init: workspace not 256-byte aligned");
    std::string why;
    for (int k = 0; k < ncases; ++k)
        if (!validate_case(lattice, storage, cases[k], why))
            return fail(nullptr, MDF_EINVAL, "mdf_init: case %d: %s", k, why.c_str());
    if (init_kind != MDF_INIT_REST) {
        if (!init_data) return fail(nullptr, MDF_EINVAL, "mdf_init: init_data is NULL");
        for (int k = 0; k < ncases; ++k)
            if (!init_data[k]) return fail(nullptr, MDF_EINVAL, "mdf_init: init_data[%d] is NULL", k);
    }
    bool has_solid = false;
    if (solid)
        for (int k = 0; k < ncases; ++k) has_solid = has_solid || solid[k] != nullptr;
    std::vector<CaseLayout> lay;
    SharedLayout shl;
    const size_t need = layout(lattice, storage, cases, ncases, has_solid, &lay, &shl);
    if (ws_bytes < need)
        return fail(nullptr, MDF_ENOMEM, "mdf_init: workspace of %zu bytes, %zu needed", ws_bytes, need);

    mdf_ctx *ctx = new mdf_ctx;
    ctx->lattice = lattice;
    ctx->shape.fuse = lat_fused_default(lattice, storage) ? 1 : 0;
    if (!lat_2d(lattice) && !lat_diag(lattice) && (storage == MDF_F16DEV || storage == MDF_BF16DEV)) {
        // one step per launch in 3D: 128 x 2 blocks without XCD bands ran
        // 0-3 % faster than 64 x 4 with bands at 128^3 and 9-12 % at 256^3
        // and 384^3 (D3Q7, FP16 and BF16)
        ctx->shape.bx = 128;
        ctx->shape.by = 2;
        ctx->shape.groups = 1;
    }
    ctx->storage = storage;
    ctx->d = lat_d(lattice);
    ctx->q = lat_q(lattice);
    ctx->ncases = ncases;
    ctx->kc.resize(ncases);
    ctx->bufs.resize(ncases);
    ctx->cur.assign(ncases, 0);
    ctx->time.assign(ncases, 0);
    ctx->snap_time.assign(ncases, -1);
    ctx->enabled.assign(ncases, 1);
    ctx->host_red.assign(mdf::kNRed, 0.0);
    char *ws = static_cast<char *>(workspace);
    ctx->batched = ncases > 1;
    ctx->any_mask = has_solid;
    ctx->d_tab = reinterpret_cast<mdf::BatchEntry *>(ws + shl.table);
    ctx->d_meta = reinterpret_cast<int *>(ws + shl.meta);
    ctx->d_tile_start = reinterpret_cast<int *>(ws + shl.tile_start);
    ctx->d_tile_start2 = reinterpret_cast<int *>(ws + shl.tile_start2);
    ctx->d_active = reinterpret_cast<int *>(ws + shl.active);
    ctx->d_results = reinterpret_cast<double *>(ws + lay[0].result);
    ctx->h_results.assign(size_t(ncases) * mdf::kNRed, 0.0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int k = 0; k < ncases; ++k) {
        ctx->kc[k] = make_kcase(lattice, storage, cases[k]);
        CaseBufs &b = ctx->bufs[k];
        b.pop[0] = ws + lay[k].pop[0];
        b.pop[1] = ws + lay[k].pop[1];
        // with obstacles in any case, every case carries link bits (zero
        // where it has no mask), so batched launches read valid memory
        b.links = has_solid ? reinterpret_cast<uint8_t *>(ws + lay[k].links) : nullptr;
        b.snap = ws + lay[k].snap;
        b.partial = reinterpret_cast<double *>(ws + lay[k].partial);
        b.result = reinterpret_cast<double *>(ws + lay[k].result);
        b.max_blocks = lay[k].max_blocks;
        hipError_t e;
        if (b.links) {
            e = mdf::launch_links(lattice, ctx->kc[k], solid[k], b.links, st);
            if (e != hipSuccess) {
                mdf_status s = device_error(nullptr, e, "mdf_init: links launch");
                delete ctx;
                return s;
            }
        }
        e = mdf::launch_init(lattice, storage, ctx->kc[k], b, 0, init_kind,
                             init_kind == MDF_INIT_REST ? nullptr : init_data[k], st);
        if (e != hipSuccess) {
            mdf_status s = device_error(nullptr, e, "mdf_init: init launch");
            delete ctx;
            return s;
        }
    }
    // Populations the next launch cannot find in the 256 MB Infinity Cache
    // are written with a non-temporal hint (measured: +3.4-4.4 % on 8192^2
    // and 256^3 grids, -23 % on a 1024^2 grid that fits the cache).
    size_t pop_total = 0;
    for (int k = 0; k < ncases; ++k)
        pop_total += 2 * size_t(lat_planes(lattice)) * size_t(ctx->kc[k].dstride) * storage_bytes(storage);
    const size_t kInfinityCacheBytes = size_t(256) << 20;
    for (int k = 0; k < ncases; ++k) ctx->kc[k].ntstore = pop_total > kInfinityCacheBytes ? 1 : 0;
    *out = ctx;
    return MDF_OK;
}

mdf_status mdf_set_launch(mdf_ctx *ctx, int32_t bx, int32_t by, int32_t groups, int32_t form)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_set_launch: ctx is NULL");
    if (bx < 32 || bx % 32 != 0 || by < 1 || bx * by > 256 || (bx * by) % 64 != 0)
        return fail(ctx, MDF_EINVAL,
                    "mdf_set_launch: need bx %% 32 == 0 and bx*by a multiple of 64 up to 256 (got %d x %d)", bx, by);
    if (groups < 0 || groups > 64) return fail(ctx, MDF_EINVAL, "mdf_set_launch: groups outside [0, 64]");
    if (form < 0 || form > 2) return fail(ctx, MDF_EINVAL, "mdf_set_launch: form must be 0, 1 or 2");
    if (form == 2 && !lat_fusable(ctx->lattice))
        return fail(ctx, MDF_EINVAL, "mdf_set_launch: two steps per launch needs a lattice with axis links");
    if (form == 1 && lat_diag(ctx->lattice))
        return fail(ctx, MDF_EINVAL, "mdf_set_launch: the vector form needs a lattice with axis links");
    ctx->shape = LaunchShape{bx, by, groups, form == 1 ? 2 : 1, form == 2 ? 1 : 0};
    drop_graphs(ctx);
    return MDF_OK;
}

static mdf_status step_impl(mdf_ctx *ctx, int32_t nsteps, uint32_t fields, void *const *out, void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_step: ctx is NULL");
    if (ctx->latched != hipSuccess) return fail(ctx, MDF_EDEVICE, "earlier device error: %s",
                                                hipGetErrorString(ctx->latched));
    if (nsteps < 0) return fail(ctx, MDF_EINVAL, "mdf_step: nsteps < 0");
    if (fields & ~(MDF_FIELD_ALL | MDF_FIELD_ACCUMULATE))
        return fail(ctx, MDF_EINVAL, "mdf_step_emit: unknown field bits");
    if (fields && !(fields & MDF_FIELD_ALL)) return fail(ctx, MDF_EINVAL, "mdf_step_emit: no fields selected");
    if (fields) {
        if (!out) return fail(ctx, MDF_EINVAL, "mdf_step_emit: out is NULL");
        for (int k = 0; k < ctx->ncases; ++k)
            if (!out[k]) return fail(ctx, MDF_EINVAL, "mdf_step_emit: out[%d] is NULL", k);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->batched) {
        std::vector<int> all;
        for (int k = 0; k < ctx->ncases; ++k)
            if (ctx->enabled[k]) all.push_back(k);
        if (all.empty()) return MDF_OK;
        mdf_status r = batch_upload(ctx, all, fields, out, st);
        if (r != MDF_OK) return r;
        return batch_steps(ctx, nsteps, false, fields, st);
    }
    for (int k = 0; k < ctx->ncases; ++k) {
        if (!ctx->enabled[k]) continue;
        mdf_status r = advance_case(ctx, k, nsteps, false, fields, fields ? out[k] : nullptr, st, nullptr);
        if (r != MDF_OK) return r;
    }
    return MDF_OK;
}

mdf_status mdf_step(mdf_ctx *ctx, int32_t nsteps, void *stream) { return step_impl(ctx, nsteps, 0, nullptr, stream); }

mdf_status mdf_step_emit(mdf_ctx *ctx, int32_t nsteps, uint32_t fields, void *const *out, void *stream)
{
    if (fields == 0) return fail(ctx, MDF_EINVAL, "mdf_step_emit: no fields selected");
    return step_impl(ctx, nsteps, fields, out, stream);
}

static mdf_status read_impl(const mdf_ctx *cctx, int32_t case_id, int mode, uint32_t fields, void *out,
                            void *stream, int *nblocks)
{
    mdf_ctx *ctx = const_cast<mdf_ctx *>(cctx);
    if (!ctx) return fail(nullptr, MDF_EINVAL, "read: ctx is NULL");
    if (ctx->latched != hipSuccess) return fail(ctx, MDF_EDEVICE, "earlier device error: %s",
                                                hipGetErrorString(ctx->latched));
    if (!case_ok(ctx, case_id)) return fail(ctx, MDF_EINVAL, "case_id %d out of range", case_id);
    if ((mode == mdf::kReadFields || mode == mdf::kReadPops) && !out)
        return fail(ctx, MDF_EINVAL, "out is NULL");
    if (mode == mdf::kReadFields && (fields == 0 || (fields & ~MDF_FIELD_ALL)))
        return fail(ctx, MDF_EINVAL, "bad field selection 0x%x", fields);
    const int k = case_id;
    if ((mode == mdf::kReadCheck || mode == mdf::kReadSums) &&
        mdf::read_blocks(ctx->kc[k], ctx->shape) > ctx->bufs[k].max_blocks)
        return fail(ctx, MDF_EINVAL, "launch grid exceeds the reduction workspace");
    const bool pull = ctx->time[k] > 0;
    hipError_t e = mdf::launch_read(ctx->lattice, ctx->storage, ctx->kc[k], ctx->bufs[k], ctx->cur[k] ^ 1, pull,
                                    mode, fields, out, ctx->shape, nblocks, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(ctx, e, "read launch");
    return MDF_OK;
}

mdf_status mdf_moments(const mdf_ctx *ctx, int32_t case_id, void *out, void *stream)
{
    return read_impl(ctx, case_id, mdf::kReadFields, MDF_FIELD_MOMENTS, out, stream, nullptr);
}

mdf_status mdf_gradients(const mdf_ctx *ctx, int32_t case_id, uint32_t fields, void *out, void *stream)
{
    return read_impl(ctx, case_id, mdf::kReadFields, fields, out, stream, nullptr);
}

mdf_status mdf_populations(const mdf_ctx *ctx, int32_t case_id, void *out, void *stream)
{
    return read_impl(ctx, case_id, mdf::kReadPops, 0, out, stream, nullptr);
}

mdf_status mdf_check(mdf_ctx *ctx, double *res, int32_t *status, void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_check: ctx is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool unstable = false;
    for (int k = 0; k < ctx->ncases; ++k) {
        int nb = 0;
        mdf_status r = read_impl(ctx, k, mdf::kReadCheck, 0, nullptr, stream, &nb);
        if (r != MDF_OK) return r;
        r = finalize_and_fetch(ctx, k, nb, st, ctx->host_red.data());
        if (r != MDF_OK) return r;
        const double rr = residual_of(ctx, k, ctx->host_red.data());
        ctx->snap_time[k] = ctx->time[k];
        const bool bad = ctx->host_red[7] != 0.0 || !std::isfinite(ctx->host_red[1]);
        unstable = unstable || bad;
        if (res) res[k] = rr;
        if (status) status[k] = bad ? 1 : 0;
    }
    if (unstable) return fail(ctx, MDF_EUNSTABLE, "mdf_check: non-finite values");
    return MDF_OK;
}

mdf_status mdf_run_steady(mdf_ctx *ctx, double tol, int32_t K, int64_t max_steps, uint32_t fields,
                          void *const *out, int32_t *case_status, int64_t *steps_taken, double *final_res,
                          void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_run_steady: ctx is NULL");
    if (!(tol > 0.0) || K < 1 || max_steps < 0) return fail(ctx, MDF_EINVAL, "mdf_run_steady: bad tol/K/max_steps");
    if (fields & ~(MDF_FIELD_ALL | MDF_FIELD_ACCUMULATE))
        return fail(ctx, MDF_EINVAL, "mdf_run_steady: unknown field bits");
    if (fields && !(fields & MDF_FIELD_ALL)) return fail(ctx, MDF_EINVAL, "mdf_run_steady: no fields selected");
    if (fields) {
        if (!out) return fail(ctx, MDF_EINVAL, "mdf_run_steady: out is NULL");
        for (int k = 0; k < ctx->ncases; ++k)
            if (!out[k]) return fail(ctx, MDF_EINVAL, "mdf_run_steady: out[%d] is NULL", k);
    }
    if (ctx->latched != hipSuccess) return fail(ctx, MDF_EDEVICE, "earlier device error: %s",
                                                hipGetErrorString(ctx->latched));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = ctx->ncases;
    std::vector<int> state(n, 2);              // 0 converged, 1 non-finite, 2 running, 3 disabled
    std::vector<double> res(n, INFINITY);
    std::vector<int64_t> start(ctx->time.begin(), ctx->time.end());
    for (int k = 0; k < n; ++k)
        if (!ctx->enabled[k]) state[k] = 3;
    // first snapshot
    for (int k = 0; k < n; ++k) {
        if (state[k] != 2) continue;
        if (ctx->snap_time[k] >= 0 && ctx->snap_time[k] == ctx->time[k]) continue;
        int nb = 0;
        mdf_status r = read_impl(ctx, k, mdf::kReadCheck, 0, nullptr, stream, &nb);
        if (r != MDF_OK) return r;
        r = finalize_and_fetch(ctx, k, nb, st, ctx->host_red.data());
        if (r != MDF_OK) return r;
        ctx->snap_time[k] = ctx->time[k];
        if (ctx->host_red[7] != 0.0) state[k] = 1;
    }
    if (ctx->batched) {
        std::vector<int> active;
        for (int k = 0; k < n; ++k)
            if (state[k] == 2) active.push_back(k);
        int64_t done = 0;
        bool need_upload = true;
        while (!active.empty() && done < max_steps) {
            if (need_upload) {
                mdf_status r = batch_upload(ctx, active, fields, out, st);
                if (r != MDF_OK) return r;
                need_upload = false;
            }
            const int chunk = int(std::min<int64_t>(K, max_steps - done));
            mdf_status r = batch_steps(ctx, chunk, true, fields, st);
            if (r != MDF_OK) return r;
            done += chunk;
            r = batch_fetch_results(ctx, st);
            if (r != MDF_OK) return r;
            std::vector<int> still;
            for (int k : active) {
                const double *red = ctx->h_results.data() + size_t(k) * mdf::kNRed;
                res[k] = residual_of(ctx, k, red);
                ctx->snap_time[k] = ctx->time[k];
                if (red[7] != 0.0 || !std::isfinite(red[1])) state[k] = 1;
                else if (res[k] < tol) state[k] = 0;
                else still.push_back(k);
            }
            if (still.size() != active.size()) need_upload = true;
            active.swap(still);
        }
    }
    bool any_running = !ctx->batched;
    while (any_running) {
        any_running = false;
        for (int k = 0; k < n; ++k) {
            if (state[k] != 2) continue;
            const int64_t done = ctx->time[k] - start[k];
            if (done >= max_steps) continue;
            const int64_t chunk = std::min<int64_t>(K, max_steps - done);
            int nb = 0;
            {
                mdf_status r = advance_case(ctx, k, chunk, true, fields, fields ? out[k] : nullptr, st, &nb);
                if (r != MDF_OK) return r;
            }
            mdf_status r = finalize_and_fetch(ctx, k, nb, st, ctx->host_red.data());
            if (r != MDF_OK) return r;
            res[k] = residual_of(ctx, k, ctx->host_red.data());
            ctx->snap_time[k] = ctx->time[k];
            if (ctx->host_red[7] != 0.0 || !std::isfinite(ctx->host_red[1])) state[k] = 1;
            else if (res[k] < tol) state[k] = 0;
            else any_running = any_running || (ctx->time[k] - start[k] < max_steps);
        }
    }
    bool unstable = false;
    for (int k = 0; k < n; ++k) {
        if (case_status) case_status[k] = state[k];
        if (steps_taken) steps_taken[k] = ctx->time[k] - start[k];
        if (final_res) final_res[k] = res[k];
        unstable = unstable || state[k] == 1;
    }
    if (unstable) return fail(ctx, MDF_EUNSTABLE, "mdf_run_steady: non-finite values");
    return MDF_OK;
}

mdf_status mdf_invariants(const mdf_ctx *cctx, int32_t case_id, double *out, void *stream)
{
    mdf_ctx *ctx = const_cast<mdf_ctx *>(cctx);
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_invariants: ctx is NULL");
    if (!out) return fail(ctx, MDF_EINVAL, "mdf_invariants: out is NULL");
    int nb = 0;
    mdf_status r = read_impl(ctx, case_id, mdf::kReadSums, 0, nullptr, stream, &nb);
    if (r != MDF_OK) return r;
    double red[mdf::kNRed];
    r = finalize_and_fetch(ctx, case_id, nb, static_cast<hipStream_t>(stream), red);
    if (r != MDF_OK) return r;
    for (int a = 0; a <= ctx->d; ++a) out[a] = red[2 + a];
    out[ctx->d + 1] = red[6];
    if (red[7] != 0.0) return fail(ctx, MDF_EUNSTABLE, "mdf_invariants: non-finite values");
    return MDF_OK;
}

mdf_status mdf_set_force_field(mdf_ctx *ctx, int32_t case_id, const void *force)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_set_force_field: ctx is NULL");
    if (!case_ok(ctx, case_id)) return fail(ctx, MDF_EINVAL, "case_id %d out of range", case_id);
    const size_t align = ctx->storage == MDF_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(force) % align != 0)
        return fail(ctx, MDF_EINVAL, "mdf_set_force_field: force not aligned to its element size");
    ctx->kc[case_id].ffield = force;
    drop_graphs(ctx);          // captured launches hold the old case parameters
    return MDF_OK;
}

mdf_status mdf_set_active(mdf_ctx *ctx, const int32_t *active)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_set_active: ctx is NULL");
    if (!active) return fail(ctx, MDF_EINVAL, "mdf_set_active: active is NULL");
    for (int k = 0; k < ctx->ncases; ++k) ctx->enabled[k] = active[k] != 0;
    return MDF_OK;
}

mdf_status mdf_autotune(mdf_ctx *ctx, int32_t trial_steps, int32_t *chosen, double *best_ms, void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_autotune: ctx is NULL");
    if (trial_steps < 1) return fail(ctx, MDF_EINVAL, "mdf_autotune: trial_steps < 1");
    static const int cand[][4] = {{64, 4, 8, 1}, {128, 2, 8, 1}, {256, 1, 8, 1}, {64, 2, 8, 1},
                                  {64, 1, 8, 1}, {64, 4, 1, 1}, {64, 4, 8, 0}, {128, 2, 8, 0},
                                  {256, 1, 8, 0}, {64, 4, 1, 0}, {128, 1, 8, 0}, {32, 8, 8, 0},
                                  {128, 2, 1, 0}, {128, 1, 1, 0}, {128, 2, 8, 2}, {64, 4, 1, 2}};
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return device_error(ctx, e, "event create");
    float best = 1e30f;
    int bi = 0;
    mdf_status r = MDF_OK;
    for (int c = 0; c < int(sizeof cand / sizeof cand[0]) && r == MDF_OK; ++c) {
        // two steps per launch: lattices with axis links
        if (cand[c][3] == 2 && !lat_fusable(ctx->lattice)) continue;
        if (cand[c][3] == 1 && lat_diag(ctx->lattice)) continue;
        r = mdf_set_launch(ctx, cand[c][0], cand[c][1], cand[c][2], cand[c][3]);
        if (r != MDF_OK) break;
        r = step_impl(ctx, 1, 0, nullptr, stream);           // warm-up (and graph capture)
        if (r != MDF_OK) break;
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            r = step_impl(ctx, trial_steps, 0, nullptr, stream);
            if (r != MDF_OK) break;
            e = hipEventRecord(e1, st);
        }
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { r = device_error(ctx, e, "autotune timing"); break; }
        if (ms < best) { best = ms; bi = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != MDF_OK) return r;
    r = mdf_set_launch(ctx, cand[bi][0], cand[bi][1], cand[bi][2], cand[bi][3]);
    if (chosen)
        for (int k = 0; k < 4; ++k) chosen[k] = cand[bi][k];
    if (best_ms) *best_ms = double(best) / trial_steps;
    return r;
}

mdf_status mdf_graph_stats(const mdf_ctx *ctx, int64_t *stats, const char **capture_error)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_graph_stats: ctx is NULL");
    if (!stats) return fail(const_cast<mdf_ctx *>(ctx), MDF_EINVAL, "mdf_graph_stats: stats is NULL");
    stats[0] = ctx->graphs_captured;
    stats[1] = ctx->graph_launches;
    stats[2] = ctx->plain_chunks;
    stats[3] = ctx->capture_failures;
    if (capture_error) *capture_error = ctx->capture_error.c_str();
    return MDF_OK;
}

mdf_status mdf_population_buffer(const mdf_ctx *ctx, int32_t case_id, int32_t which, void **ptr, size_t *bytes)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_population_buffer: ctx is NULL");
    mdf_ctx *c = const_cast<mdf_ctx *>(ctx);
    if (!case_ok(ctx, case_id)) return fail(c, MDF_EINVAL, "case_id %d out of range", case_id);
    if (which != 0 && which != 1) return fail(c, MDF_EINVAL, "mdf_population_buffer: which must be 0 or 1");
    if (!ptr || !bytes) return fail(c, MDF_EINVAL, "mdf_population_buffer: NULL output");
    *ptr = ctx->bufs[case_id].pop[which == 0 ? ctx->cur[case_id] : ctx->cur[case_id] ^ 1];
    *bytes = size_t(lat_planes(ctx->lattice)) * size_t(ctx->kc[case_id].dstride) * storage_bytes(ctx->storage);
    return MDF_OK;
}

int64_t mdf_time(const mdf_ctx *ctx, int32_t case_id)
{
    if (!ctx || !case_ok(ctx, case_id)) return -1;
    return ctx->time[case_id];
}

const char *mdf_last_error(const mdf_ctx *ctx)
{
    if (!ctx) return g_last_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

// ----------------------------------------------------------------- checkpoint

namespace {

struct StateHeader {
    char magic[8];          // "MDFSTAT1"
    int32_t lattice, storage, ncases, reserved;
    uint64_t total_bytes;
};

struct StateCase {
    int32_t nx, ny, nz, pitch;
    int64_t time, snap_time;
    int32_t enabled, reserved;
    uint64_t pop_bytes, snap_bytes;     // one population buffer; the velocity snapshot
};

const char kStateMagic[8] = {'M', 'D', 'F', 'S', 'T', 'A', 'T', '1'};

size_t case_pop_bytes(const mdf_ctx *ctx, int k)
{
    return size_t(lat_planes(ctx->lattice)) * size_t(ctx->kc[k].dstride) * storage_bytes(ctx->storage);
}

size_t case_snap_bytes(const mdf_ctx *ctx, int k)
{
    const KCase &p = ctx->kc[k];
    return size_t(ctx->d) * size_t(p.nx) * p.ny * p.nz * compute_bytes(ctx->storage);
}

size_t state_bytes(const mdf_ctx *ctx)
{
    size_t n = sizeof(StateHeader) + size_t(ctx->ncases) * sizeof(StateCase);
    for (int k = 0; k < ctx->ncases; ++k) n += 2 * case_pop_bytes(ctx, k) + case_snap_bytes(ctx, k);
    return n;
}

}  // namespace

extern "C" {

size_t mdf_state_size(const mdf_ctx *ctx)
{
    return ctx ? state_bytes(ctx) : 0;
}

mdf_status mdf_save(mdf_ctx *ctx, void *dst, size_t bytes, void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_save: ctx is NULL");
    if (ctx->latched != hipSuccess) return fail(ctx, MDF_EDEVICE, "earlier device error: %s",
                                                hipGetErrorString(ctx->latched));
    if (!dst) return fail(ctx, MDF_EINVAL, "mdf_save: dst is NULL");
    const size_t need = state_bytes(ctx);
    if (bytes < need) return fail(ctx, MDF_EINVAL, "mdf_save: %zu bytes given, %zu needed", bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<char> head(sizeof(StateHeader) + size_t(ctx->ncases) * sizeof(StateCase));
    StateHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kStateMagic, 8);
    h.lattice = ctx->lattice;
    h.storage = ctx->storage;
    h.ncases = ctx->ncases;
    h.total_bytes = need;
    std::memcpy(head.data(), &h, sizeof h);
    char *out = static_cast<char *>(dst);
    size_t off = head.size();
    for (int k = 0; k < ctx->ncases; ++k) {
        StateCase c;
        std::memset(&c, 0, sizeof c);
        c.nx = ctx->kc[k].nx;
        c.ny = ctx->kc[k].ny;
        c.nz = ctx->kc[k].nz;
        c.pitch = ctx->kc[k].pitch;
        c.time = ctx->time[k];
        c.snap_time = ctx->snap_time[k];
        c.enabled = ctx->enabled[k];
        c.pop_bytes = case_pop_bytes(ctx, k);
        c.snap_bytes = case_snap_bytes(ctx, k);
        std::memcpy(head.data() + sizeof h + size_t(k) * sizeof c, &c, sizeof c);
        // the buffer holding f*(t) first, then the one the read kernels pull from
        const int cur = ctx->cur[k];
        hipError_t e = hipMemcpyAsync(out + off, ctx->bufs[k].pop[cur], c.pop_bytes, hipMemcpyDefault, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + off + c.pop_bytes, ctx->bufs[k].pop[cur ^ 1], c.pop_bytes, hipMemcpyDefault, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + off + 2 * c.pop_bytes, ctx->bufs[k].snap, c.snap_bytes, hipMemcpyDefault, st);
        if (e != hipSuccess) return device_error(ctx, e, "mdf_save copy");
        off += 2 * c.pop_bytes + c.snap_bytes;
    }
    hipError_t e = hipMemcpyAsync(out, head.data(), head.size(), hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);      // `head` is a host temporary
    if (e != hipSuccess) return device_error(ctx, e, "mdf_save header");
    return MDF_OK;
}

mdf_status mdf_load(mdf_ctx *ctx, const void *src, size_t bytes, void *stream)
{
    if (!ctx) return fail(nullptr, MDF_EINVAL, "mdf_load: ctx is NULL");
    if (ctx->latched != hipSuccess) return fail(ctx, MDF_EDEVICE, "earlier device error: %s",
                                                hipGetErrorString(ctx->latched));
    if (!src) return fail(ctx, MDF_EINVAL, "mdf_load: src is NULL");
    const size_t need = state_bytes(ctx);
    const size_t head_bytes = sizeof(StateHeader) + size_t(ctx->ncases) * sizeof(StateCase);
    if (bytes < head_bytes) return fail(ctx, MDF_EINVAL, "mdf_load: %zu bytes is not a saved state", bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<char> head(head_bytes);
    hipError_t e = hipMemcpyAsync(head.data(), src, head_bytes, hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error(ctx, e, "mdf_load header");
    StateHeader h;
    std::memcpy(&h, head.data(), sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(ctx, MDF_EINVAL, "mdf_load: not a saved state");
    if (h.lattice != ctx->lattice || h.storage != ctx->storage || h.ncases != ctx->ncases)
        return fail(ctx, MDF_EINVAL, "mdf_load: saved with lattice %d, storage %d, %d cases; context has %d, %d, %d",
                    h.lattice, h.storage, h.ncases, ctx->lattice, ctx->storage, ctx->ncases);
    if (h.total_bytes != need || bytes < need)
        return fail(ctx, MDF_EINVAL, "mdf_load: state of %llu bytes (%zu given), context needs %zu",
                    (unsigned long long)h.total_bytes, bytes, need);
    std::vector<StateCase> cs(ctx->ncases);
    for (int k = 0; k < ctx->ncases; ++k) {
        std::memcpy(&cs[k], head.data() + sizeof h + size_t(k) * sizeof(StateCase), sizeof(StateCase));
        const StateCase &c = cs[k];
        const KCase &p = ctx->kc[k];
        if (c.nx != p.nx || c.ny != p.ny || c.nz != p.nz || c.pitch != p.pitch ||
            c.pop_bytes != case_pop_bytes(ctx, k) || c.snap_bytes != case_snap_bytes(ctx, k))
            return fail(ctx, MDF_EINVAL, "mdf_load: case %d was %d x %d x %d, context has %d x %d x %d", k, c.nx,
                        c.ny, c.nz, p.nx, p.ny, p.nz);
    }
    const char *in = static_cast<const char *>(src);
    size_t off = head_bytes;
    for (int k = 0; k < ctx->ncases; ++k) {
        const StateCase &c = cs[k];
        e = hipMemcpyAsync(ctx->bufs[k].pop[0], in + off, c.pop_bytes, hipMemcpyDefault, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->bufs[k].pop[1], in + off + c.pop_bytes, c.pop_bytes, hipMemcpyDefault, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->bufs[k].snap, in + off + 2 * c.pop_bytes, c.snap_bytes, hipMemcpyDefault, st);
        if (e != hipSuccess) return device_error(ctx, e, "mdf_load copy");
        off += 2 * c.pop_bytes + c.snap_bytes;
        ctx->cur[k] = 0;
        ctx->time[k] = c.time;
        ctx->snap_time[k] = c.snap_time;
        ctx->enabled[k] = c.enabled ? 1 : 0;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error(ctx, e, "mdf_load synchronize");
    drop_graphs(ctx);            // captured launches name the old buffer parity
    return MDF_OK;
}

mdf_status mdf_destroy(mdf_ctx *ctx)
{
    if (ctx) drop_graphs(ctx);
    delete ctx;
    return MDF_OK;
}

}  // extern "C"
