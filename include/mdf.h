/*
 * mdf.h -- C ABI of the MI355X (gfx950) library for the multiple-
 * distribution-function MRT lattice Boltzmann method of Chai, Shi & Zhan,
 * "Multiple-distribution-function lattice Boltzmann method for convection-
 * diffusion-system based incompressible Navier-Stokes equations"
 * (arXiv 2108.08591).
 *
 * The method treats the incompressible Navier-Stokes equations as d+1 coupled
 * convection-diffusion equations (eq. 2-2) for ubar = (rho0, u_1..u_d) and
 * advances one distribution set per equation with the evolution of Remark I
 * (eq. 3-21):
 *     f_{i,a}(x + c_i, t + 1) = f_{i,a} - sum_k L_{ik}(f_{k,a} - f^eq_{k,a}) + w_i Fbar_a
 * on the D2Q5 (eq. d2q5) or D3Q7 (eq. d3q7) lattice, with L = M^{-1} S_d M
 * (eq. 4-1..4-3), the linear equilibrium of eq. 2-4, the pressure of eq. 3-15
 * and the local velocity gradient, divergence, strain rate, stress and
 * vorticity of eq. 3-16..3-19.  Lattice units: dx = dt = c = 1.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns an mdf_status; nothing is thrown across the ABI.
 *   Arguments are validated on the host before any launch; a rejected call
 *   launches nothing and leaves the context unchanged.  The message of the
 *   last failure of a context is available from mdf_last_error().
 * - Device memory is owned by the caller: the workspace, masks, initial
 *   data and output buffers are device pointers the caller allocates (e.g.
 *   torch tensors) and keeps alive until the stream has passed the call.
 *   The library never allocates device memory; it owns only the host-side
 *   context, released by mdf_destroy().
 * - Work is enqueued on the HIP stream passed as `stream` (hipStream_t;
 *   NULL = the null stream).  Only mdf_run_steady, mdf_check and
 *   mdf_invariants wait for the device.
 * - Compute dtype: FP64 for MDF_F64 storage, FP32 for every other storage.
 *   All field inputs and outputs are in the compute dtype, contiguous,
 *   channel-major: out[ch][z][y][x] with x fastest and no padding.
 * - Time: mdf_init sets time 0; mdf_step(n) advances it by n.  Fields
 *   reported "at time t" are computed from the pre-collision populations
 *   f(x, t) (the state right after streaming into time t).
 * - Calls that overlap on one context race; contexts are independent.
 */
#ifndef MDF_H
#define MDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDF_OK = 0,
    MDF_EINVAL = -1,     /* invalid argument (nothing launched)            */
    MDF_ENOMEM = -2,     /* workspace too small                            */
    MDF_EDEVICE = -3,    /* HIP runtime error (latched in the context)     */
    MDF_EUNSTABLE = -4,  /* non-finite values found at a check             */
    MDF_ESTATE = -5      /* call not valid in the context's current state  */
} mdf_status;

/* Lattices (eq. d2q5, eq. d3q7, eq. d2q4, eq. d3q6).  MDF_D2Q5 / MDF_D3Q7
 * store all d + 1 distribution sets a = 0..d of eq. 2-2 (ubar_0 = rho0,
 * ubar_a = u_a).  The *_V variants store only the d velocity sets a = 1..d
 * (Remark IV: the set a = 0 advects rho0 passively and no other quantity
 * reads it), moving d/(d+1) of the bytes per step; their velocity sets, P
 * and every derived field are identical to the full form's, and ubar_0 reads
 * as the constant rho0.  Populations (mdf_populations, MDF_INIT_POPULATIONS)
 * then have d sets, a = 1..d.
 * MDF_D2Q4 (cs^2 = 1/2) and MDF_D3Q6 (cs^2 = 1/3) have no rest population
 * (4/5 and 6/7 of the bytes of D2Q5 and D3Q7); their populations are
 * ordered as the columns of eq. d2q4 (+x, +y, -x, -y) and eq. d3q6 (+x, -x,
 * +y, -y, +z, -z).  The paper prints no collision matrix for them; the one
 * used keeps the structure of eq. 4-1..4-3: s0 on the conserved moment, s1
 * on the d first moments and s2 on every other moment (xx - yy on D2Q4;
 * 2xx - yy - zz and yy - zz on D3Q6), so the viscosity is
 * nu = (1/s1 - 1/2) cs^2 with the lattice's own cs^2.
 * MDF_D2Q9 and MDF_D3Q15 (cs^2 = 1/3) add diagonal links, in the column
 * order of eq. d2q9 and eq. d3q15.  Their collision relaxes every moment
 * odd under c -> -c with s1 and every even one with s2 (the structure of
 * eq. 4-3 carried to the larger moment sets).  A diagonal link whose
 * upstream point lies behind two or three wall faces takes the first of them
 * in the order x, y, z.  They run one node per thread (form 0) only.
 * MDF_D2Q9_Q5 and MDF_D3Q15_Q7 take a lattice per set (allowed by the
 * remark after eq. d3q15): the velocity sets a = 1..d on D2Q9 / D3Q15 as
 * above, the set a = 0, which only advects rho0, on D2Q5 / D3Q7 with that
 * lattice's weights and cs^2.  The D2Q5 / D3Q7 velocities are the first five
 * / seven columns of the larger lattice, so a set-0 population keeps its
 * direction index.  One buffer holds 5 + 2 x 9 = 23 (2D) or 7 + 3 x 15 = 52
 * (3D) population planes, set 0's first.  Populations (mdf_populations,
 * MDF_INIT_POPULATIONS) keep the [set][dir] layout of the full lattice, the
 * set a = 0 padded with zeros at directions 2d+1 .. q-1 (read back as zero,
 * ignored on input).  Velocity sets, P and every derived field follow the
 * D2Q9 / D3Q15 lattice.  Form 0 only. */
typedef enum {
    MDF_D2Q5 = 0, MDF_D3Q7 = 1, MDF_D2Q5_V = 2, MDF_D3Q7_V = 3,
    MDF_D2Q4 = 4, MDF_D3Q6 = 5, MDF_D2Q4_V = 6, MDF_D3Q6_V = 7,
    MDF_D2Q9 = 8, MDF_D3Q15 = 9, MDF_D2Q9_V = 10, MDF_D3Q15_V = 11,
    MDF_D2Q9_Q5 = 12, MDF_D3Q15_Q7 = 13
} mdf_lattice;

/* Storage of the populations.  MDF_F16DEV / MDF_BF16DEV keep
 * (f - f_rest) / u_ref in 16 bits (round to nearest even on store), with
 * f_rest_{i,0} = w_i rho0 and f_rest_{i,a>=1} = 0, and collide in FP32. */
typedef enum { MDF_F64 = 0, MDF_F32 = 1, MDF_F16DEV = 2, MDF_BF16DEV = 3 } mdf_storage;

typedef enum { MDF_PERIODIC = 0, MDF_WALL = 1 } mdf_bc;

/* Field selection bits.  Channels are written in the order of the bits:
 *   MOMENTS: ubar_0 .. ubar_d (eq. 2-7), then P (eq. 3-15)      d + 2
 *   GRAD:    d u_a / d x_b at (a-1)*d + b (eq. 3-16)            d * d
 *   DIV:     div u (eq. 3-16a)                                  1
 *   STRAIN:  S (eq. 3-17), upper triangle row by row            d(d+1)/2
 *            (xx, xy, yy) in 2D, (xx, xy, xz, yy, yz, zz) in 3D
 *   STRESS:  sigma (eq. 3-17a), same order as STRAIN            d(d+1)/2
 *   VORT:    omega = dv/dx - du/dy in 2D; curl u in 3D          1 or 3
 *            (eq. 3-18 with eq. 3-19)                                    */
#define MDF_FIELD_MOMENTS 0x01u
#define MDF_FIELD_GRAD 0x02u
#define MDF_FIELD_DIV 0x04u
#define MDF_FIELD_STRAIN 0x08u
#define MDF_FIELD_STRESS 0x10u
#define MDF_FIELD_VORT 0x20u
#define MDF_FIELD_ALL 0x3fu
/* Modifier of a field selection for mdf_step_emit and mdf_run_steady:
 * every step adds its fields to out[case] instead of overwriting them, in
 * the compute dtype, one rounding per step (out <- out + field(t)), so that
 * after n steps out holds the sum over the n new times (their time mean
 * times n); the caller initialises out.  Solid nodes add nothing.  Two-step
 * launches contribute both of their steps.  The selected fields of each
 * step are bitwise those of a one-step launch, so the sum is bitwise the
 * sequential sum of the per-step fields. */
#define MDF_FIELD_ACCUMULATE 0x40u

/* Initial state kinds for mdf_init (init_data[case] is a device pointer in
 * the compute dtype, channel-major, unpadded):
 *   REST:        P = 0, u = 0, ubar_0 = rho0; init_data ignored.
 *   FIELDS:      [P][u_1]..[u_d]; f = f^eq (eq. 2-4).
 *   FIELDS_GRAD: [P][u_1]..[u_d][grad u: d*d, (a-1)*d + b]; f = f^eq + f^ne
 *                with f^ne_{i,a} = -(1/s1) w_i c_i . grad u_a, which is the
 *                inverse of eq. 3-16 (the set a = 0 gets none).
 *   POPULATIONS: f(x, 0) itself, [set a][direction i][z][y][x]. */
typedef enum {
    MDF_INIT_REST = 0,
    MDF_INIT_FIELDS = 1,
    MDF_INIT_FIELDS_GRAD = 2,
    MDF_INIT_POPULATIONS = 3
} mdf_init_kind;

/* One case (lattice units).  Velocity directions are ordered
 *   D2Q5: 0, +x, +y, -x, -y          (eq. d2q5)
 *   D3Q7: 0, +x, -x, +y, -y, +z, -z  (eq. d3q7)                        */
/* Forcing scheme of a case.
 *   MDF_FORCING_PLAIN: the diffusive-scaling update of Remark I (eq. 3-21),
 *     F_{i,a} = w_i Fbar_a added once, ubar_a = sum_i f_{i,a} (eq. 2-7).
 *     Used for all of the paper's numerics.  (Scheme I, eq. 2-3b, is the
 *     same update for forces that do not change in time.)
 *   MDF_FORCING_SCHEME2: Scheme II (eq. 2-3c): the stored populations are
 *     fbar = f - F/2, updated with (I - L/2) F, and ubar_a = sum_i fbar_{i,a}
 *     + Fbar_a / 2 (eq. 2-7a); P by eq. 3-15 with fbar in place of f.  The
 *     velocity gradient (eq. 3-16) is unchanged: F_{i,a} has no first moment.
 *     Initial states from fields are shifted by -F/2 so that eq. 2-7a gives
 *     back the given velocity. */
typedef enum { MDF_FORCING_PLAIN = 0, MDF_FORCING_SCHEME2 = 1 } mdf_forcing;

typedef struct {
    int32_t nx, ny, nz;     /* nodes per axis; nz = 1 for D2Q5             */
    double s0, s1, s2;      /* S_d = diag(s0, s1.., s2..) (eq. 4-3); 0 < s1 < 2;
                               s2 <= 0 selects 8(2 - s1)/(8 - s1); the
                               viscosity is nu = (1/s1 - 1/2) cs^2 (eq. 3-13a) */
    int32_t bc[6];          /* faces -x,+x,-y,+y,-z,+z: MDF_PERIODIC or MDF_WALL;
                               periodic faces come in pairs                */
    double wall_u[6][3];    /* velocity of each wall face                  */
    double force[3];        /* uniform body force F_a (eq. 2-1b, eq. 2-6)   */
    double R;               /* uniform mass source R (eq. 2-1a); Fbar_0 = R */
    double rho0;            /* constant density (eq. 2-2, eq. 3-17a); > 0  */
    double u_ref;           /* 16-bit storage scale; <= 0 selects 1        */
    int32_t forcing;        /* mdf_forcing: how F and R enter the update    */
} mdf_case;

typedef struct mdf_ctx mdf_ctx;

/* Bytes of device workspace that mdf_init needs for these cases (0 if the
 * arguments are invalid).  has_solid != 0 reserves room for obstacle masks. */
size_t mdf_workspace_size(mdf_lattice lattice, mdf_storage storage, const mdf_case *cases,
                          int32_t ncases, int32_t has_solid);

/* Create a context over `ncases` independent cases and set time 0.
 *   workspace/ws_bytes: caller-owned device memory of at least
 *       mdf_workspace_size() bytes, 256-byte aligned, kept until mdf_destroy.
 *   solid: NULL, or per case a device uint8 mask [z][y][x] (non-zero =
 *       solid node) or NULL; links into solid nodes follow the halfway wall
 *       rule with zero wall velocity.  Copied; need not outlive the call.
 *   init_kind/init_data: see mdf_init_kind; init_data is NULL for REST or
 *       holds one device pointer per case.  Read before the call returns on
 *       the stream's timeline.
 * The wall rule on a link from behind a wall face or from a solid node is
 * the halfway anti-bounce-back of Section 4 (formula not printed there):
 *   a >= 1: f_{i,a}(x, t+1) = -f*_{ibar,a}(x, t) + 2 w_i U_{w,a}
 *   a = 0 : f_{i,0}(x, t+1) =  f*_{ibar,0}(x, t)
 * When the population buffers of all cases together exceed 256 MB (the
 * Infinity Cache), the step kernels write populations with a non-temporal
 * hint; results are the same either way.
 * Size limits per case: at most 2e9 stored populations, and every stored
 * population plane (rows padded to 128 bytes) and every field channel
 * within 4 GiB; mdf_workspace_size and mdf_init refuse larger cases.
 * Errors: MDF_EINVAL (bad lattice/storage/sizes/rates/bc pairing/pointers),
 * MDF_ENOMEM (ws_bytes too small), MDF_EDEVICE. */
mdf_status mdf_init(mdf_ctx **out, mdf_lattice lattice, mdf_storage storage,
                    const mdf_case *cases, int32_t ncases, void *workspace, size_t ws_bytes,
                    const uint8_t *const *solid, int32_t init_kind,
                    const void *const *init_data, void *stream);

/* Advance every case by nsteps time steps of eq. 3-21 (fused pull
 * streaming, wall rule, moments, equilibrium, MRT collision and forcing).
 * A context of several cases advances all of them in one persistent launch
 * per step over the flattened (case, tile) list; K-step chunks on a
 * non-null stream are captured once as a HIP graph and replayed.  The
 * results are bitwise those of one context per case with the same launch
 * shape. */
mdf_status mdf_step(mdf_ctx *ctx, int32_t nsteps, void *stream);

/* As mdf_step, and every step also writes the selected fields (MDF_FIELD_*)
 * at the new time into out[case] (channel-major, compute dtype, overwritten
 * each step: on return they hold the fields at the final time; with
 * MDF_FIELD_ACCUMULATE every step adds them instead).  MDF_EINVAL for
 * unknown bits or no field selected. */
mdf_status mdf_step_emit(mdf_ctx *ctx, int32_t nsteps, uint32_t fields, void *const *out,
                         void *stream);

/* ubar_0 .. ubar_d and P at the current time (eq. 2-7, eq. 3-15) into `out`
 * (d + 2 channels).  Bitwise equal to MDF_FIELD_MOMENTS of mdf_step_emit. */
mdf_status mdf_moments(const mdf_ctx *ctx, int32_t case_id, void *out, void *stream);

/* The fields selected by `fields` at the current time (eq. 3-16..3-19) into
 * `out`.  Bitwise equal to the same selection from mdf_step_emit. */
mdf_status mdf_gradients(const mdf_ctx *ctx, int32_t case_id, uint32_t fields, void *out,
                         void *stream);

/* Pre-collision populations f(x, t) at the current time into `out`,
 * [set][direction][z][y][x], compute dtype. */
mdf_status mdf_populations(const mdf_ctx *ctx, int32_t case_id, void *out, void *stream);

/* Residual check, waits for the device.  Computes, per case, over fluid
 * nodes and in FP64:
 *   res[c] = |u(t) - u(t_prev)|_2 / ((t - t_prev) |u(t)|_2)
 * against the velocity snapshot of the previous check (t_prev; +inf on the
 * first check), then stores u(t) as the new snapshot.  Sets status[c] to 1
 * when a non-finite value was seen.  res/status: host arrays of ncases, or
 * NULL.  Returns MDF_EUNSTABLE if any case is non-finite. */
mdf_status mdf_check(mdf_ctx *ctx, double *res, int32_t *status, void *stream);

/* Run until every case reaches res < tol (the residual of mdf_check,
 * evaluated every K steps inside the last step of each K-step chunk), goes
 * non-finite, or max_steps steps were taken.  Waits for the device once per
 * chunk.  fields/out: as mdf_step_emit (every step writes the selected
 * fields), or 0/NULL.  case_status (host, ncases or NULL): 0 converged,
 * 1 non-finite, 2 not converged, 3 disabled (mdf_set_active).  steps_taken/final_res: host arrays of
 * ncases or NULL.  Cases that converge stop advancing; the others continue.
 * Returns MDF_EUNSTABLE if any case went non-finite. */
mdf_status mdf_run_steady(mdf_ctx *ctx, double tol, int32_t K, int64_t max_steps,
                          uint32_t fields, void *const *out, int32_t *case_status,
                          int64_t *steps_taken, double *final_res, void *stream);

/* Global sums over fluid nodes at the current time, in FP64, host output
 * of d + 2 doubles: sum ubar_a for a = 0..d, then sum_{a>=1} J_{a,a} with
 * J_{a,b} = sum_i c_{i,b} f_{i,a}.  Waits for the device. */
mdf_status mdf_invariants(const mdf_ctx *ctx, int32_t case_id, double *out, void *stream);

/* Launch shape of the step and read kernels: tiles of bx (a multiple of 32)
 * by by threads, bx * by a multiple of 64 up to 256 (whole wavefronts), and
 * `groups` > 1 hands the tiles out in that many contiguous bands, one per
 * XCD (8 on MI355X), so neighbouring tiles share an L2; 0 or 1 keeps plain
 * order.  `form` selects the step kernel:
 *   0  one node per thread;
 *   1  vector: each thread of the step kernels owns consecutive x-nodes (2
 *      for MDF_STORAGE_F64, 4 for the other storages), read and written as one
 *      16-byte (8-byte for the 16-bit storages) access per plane;
 *   2  two steps per launch (the lattices with axis links only: D2Q5, D2Q4,
 *      D3Q7, D3Q6 and their *_V forms).  2D: tiles of 64 x 4/8 nodes
 *      (FP64/other storages) take one step on the tile and a one-node halo
 *      into LDS and the second from LDS.  3D: tiles of 32 x 4 (FP64), 32 x 8
 *      (FP32) or 64 x 4 (16-bit) nodes walk a
 *      chunk of z-planes, keeping the intermediate state of three planes in
 *      LDS.  Either way the state crosses HBM once per two steps.  mdf_step,
 *      mdf_step_emit and mdf_run_steady run pairs of steps this way and the
 *      last step of each call (and of each K-step chunk) as form 0 with these
 *      bx, by; batched 3D contexts run every step as form 0.
 * The read kernels always use one node per thread.  Default 64 x 4, 8
 * groups, form 2 on the axis-link lattices (in 3D with FP64 and FP32
 * storage) and form 0 elsewhere; 3D axis-link lattices with 16-bit storage
 * default to 128 x 2, one group, form 0.
 * MDF_EINVAL otherwise (also forms 1 and 2 on D2Q9 / D3Q15).  Any shape
 * and form give bitwise identical populations and fields; only the
 * summation order of the FP64 sums of mdf_check, mdf_run_steady and
 * mdf_invariants follows it. */
mdf_status mdf_set_launch(mdf_ctx *ctx, int32_t bx, int32_t by, int32_t groups, int32_t form);

/* Checkpoint and resume.  The state of a context at its current time is
 * both population buffers of every case (f*(t), and f*(t-1) that the read
 * calls pull f(t) from), the time, the residual snapshot of mdf_check and
 * the active flags, with a self-describing header.  The case parameters
 * (rates, forces, walls, masks, a force field) are not part of it: they are
 * those of the context it is loaded into, which must have the same lattice,
 * storage and grids.
 *   mdf_state_size: bytes of that state (0 for NULL).
 *   mdf_save: writes it to dst, device memory or pinned host memory of at
 *       least mdf_state_size() bytes, in stream order; returns after the
 *       stream has passed the copies.
 *   mdf_load: restores a state written by mdf_save from src (device or
 *       pinned host memory, `bytes` long); steps and reads after it are
 *       bitwise those the saved context would have produced.  Returns after
 *       the copies; src may then be freed.
 * MDF_EINVAL for NULL pointers, a short buffer, a blob that is not a saved
 * state or one saved from a different lattice, storage or grid. */
size_t mdf_state_size(const mdf_ctx *ctx);
mdf_status mdf_save(mdf_ctx *ctx, void *dst, size_t bytes, void *stream);
mdf_status mdf_load(mdf_ctx *ctx, const void *src, size_t bytes, void *stream);

/* Per-node force (eq. 2-6 with a space-dependent F, as in the four-roll
 * mill of Section 4.2) for case `case_id`: F_b(x) at force[b * nodes + node]
 * for b = 0..d-1, node = (z * ny + y) * nx + x, in the compute dtype (double
 * for MDF_STORAGE_F64, float otherwise), added to the case's uniform force
 * in the collision of every later step.  `force` is caller-owned device
 * memory that must stay valid while the context steps; NULL removes it.  The
 * pointer is read by the kernels, not copied.  MDF_EINVAL on a bad case or a
 * misaligned pointer. */
mdf_status mdf_set_force_field(mdf_ctx *ctx, int32_t case_id, const void *force);

/* Enable or disable cases.  Disabled cases are skipped by mdf_step,
 * mdf_step_emit, mdf_run_steady and mdf_autotune: their populations and
 * time stay unchanged (a disabled case gets status 3 from mdf_run_steady).
 * active: host int32[ncases], non-zero = enabled.  All cases start enabled.
 * Read-outs (mdf_moments, mdf_gradients, ...) work on any case. */
mdf_status mdf_set_active(mdf_ctx *ctx, const int32_t *active);

/* Choose the launch shape of this context by timing candidate shapes
 * (vector tiles 64x4, 128x2, 256x1, 64x2, 64x1 with XCD bands and 64x4
 * without; one-node tiles 64x4, 128x2, 256x1, 128x1, 32x8 with bands and
 * 64x4, 128x2, 128x1 without; for lattices with axis links also two steps
 * per launch with and without bands) on `trial_steps` real steps each and
 * keeping the
 * fastest.  Every case advances by (trial_steps + 1) steps per candidate
 * tried (results are bitwise independent of the shape).  chosen: host
 * int[4] (bx, by, groups, form) or NULL; best_ms: host double, time per
 * step, or NULL.  Waits for the device. */
mdf_status mdf_autotune(mdf_ctx *ctx, int32_t trial_steps, int32_t *chosen, double *best_ms,
                        void *stream);

/* How the batched steps of this context were launched (the persistent,
 * graph-captured launch of a multi-case context; see mdf_step).  stats:
 * host int64[4] receiving
 *   [0] K-step chunks captured as HIP graphs,
 *   [1] chunks run by replaying a captured graph,
 *   [2] chunks run as plain launches (the null stream, chunks of fewer
 *       than 4 steps, or after a failed capture),
 *   [3] captures that failed; the context then uses plain launches for
 *       the rest of its life, with the same results.
 * capture_error (or NULL): receives the HIP message of the last failed
 * capture ("" if none), valid until the next call on the context.
 * Single-case contexts launch per step and report zeros.  MDF_EINVAL on
 * NULL arguments. */
mdf_status mdf_graph_stats(const mdf_ctx *ctx, int64_t *stats, const char **capture_error);

/* Device address and size in bytes of one population buffer of a case, in
 * the storage layout [set][direction][z][y][row pitch]: rows padded to 128
 * bytes, each (set, direction) plane followed by a gap of 2304 bytes (plane
 * stride = bytes / number of planes).  The ping-pong pair is that of the pull
 * scheme of eq. 3-21.  which = 0: the buffer holding the
 * post-collision state f*(t) that the next step reads; which = 1: the other
 * one, which the next step overwrites and from which the read calls
 * (mdf_moments, mdf_gradients, mdf_populations, mdf_check) pull f(t).  The
 * memory stays the caller's workspace.  A caller may overwrite buffer 1
 * before a call to mdf_step or mdf_step_emit (no step reads it before
 * writing it), but not before a read call, nor before mdf_run_steady, which
 * begins with a read unless mdf_check ran at the current time.  Meant for
 * inspection and tests.  MDF_EINVAL on a bad case, `which` or NULL output. */
mdf_status mdf_population_buffer(const mdf_ctx *ctx, int32_t case_id, int32_t which, void **ptr,
                                 size_t *bytes);

/* Current time of a case (steps taken since mdf_init; cases stopped by
 * mdf_run_steady stay at their stopping time).  -1 on a bad argument. */
int64_t mdf_time(const mdf_ctx *ctx, int32_t case_id);

/* Message of the last failed call on this context ("" if none).  Valid
 * until the next call on the context.  ctx may be NULL (last failure of
 * mdf_init / mdf_workspace_size on this thread). */
const char *mdf_last_error(const mdf_ctx *ctx);

/* Release the host-side context.  The workspace stays the caller's. */
mdf_status mdf_destroy(mdf_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MDF_H */
