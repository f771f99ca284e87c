/*
 * rtm.h - C ABI of librtm: acoustic finite-difference modeling and reverse
 * time migration with random boundaries and source-wavefield
 * reconstruction, for AMD Instinct MI355X (gfx950).
 *
 * Method: Barbosa & Coutinho, "Seismic Modeling and Migration with Random
 * Boundaries on the NEC SX-Aurora TSUBASA", arXiv 2204.03380.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named "device" are HIP device allocations owned by the caller;
 *    pointers named "host" are ordinary host memory owned by the caller and
 *    read only during the call.  The library never allocates, frees or
 *    retains device memory: scratch comes from the caller's workspace `ws`
 *    (size from rtm_workspace_bytes, base aligned to 256 bytes).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is queued
 *    asynchronously on it; outputs are valid after the stream completes.
 *    rtm_model_shot, rtm_rtm_shot and rtm_model_shot_vjp synchronise the
 *    stream once, before their first propagation kernel, after uploading
 *    their acquisition tables and (unless RTM_F_SKIP_CHECK) reading back the
 *    velocity range for the stability and finiteness check.
 *  - Grids: interior extents nx, ny, nz (ny = 1 in 2-D), spacing h in
 *    metres, a random boundary of nb cells on every face.  Padded extents
 *    are NX = nx + 2nb, NZ = nz + 2nb, NY = ny + 2nb (3-D) or 1 (2-D).
 *    Dense fields are row-major [NZ][NY][NX] (x fastest); interior-sized
 *    fields are [nz][ny][nx].  Outside the padded grid the wavefield is zero
 *    (the Dirichlet condition stated with Eq. (1)).  A padded field, with the
 *    library's internal row and plane padding, must hold fewer than 2^31
 *    floats (about 2.0e9 cells; 1250^3 fits, 1300^3 does not): larger grids
 *    are refused with RTM_EINVAL, so cell offsets always fit 32 bits.
 *  - Positions are float triples (x, y, z) in interior grid units, 0-based,
 *    relative to interior cell (0, 0, 0); y is ignored in 2-D.  Off-grid
 *    positions use multilinear interpolation weights for both injection and
 *    sampling.  Every position must lie inside the interior (RTM_ERANGE).
 *  - Time: nt steps of dt seconds; the wavelet has nt samples w[0..nt-1];
 *    traces are [nrec][nt + 1] (time fastest), sample n taken at t = n dt,
 *    as the seismogram of Sec. 3 has N_rec x (N_t + 1) entries.
 *  - Discretisation (Sec. 3): 2nd order in time, 8th order in space:
 *      p^{n+1} = 2 p^n - p^{n-1} + (v dt)^2 (L_h p^n + w^n delta_s / h^d)
 *    with L_h the 9-point 8th-order Laplacian and delta_s the interpolated
 *    source.  The source enters with a positive sign (the polarity of -f in
 *    Eq. (1)); images do not depend on this choice.
 *  - Errors: every entry point returns RTM_OK (0) or a negative status.  All
 *    argument checks run on the host before any work is queued, so on an
 *    argument error nothing was launched; outputs are unspecified after any
 *    error.  rtm_last_error() describes the last failure of the calling
 *    thread.  No C++ exception crosses this interface.
 */
#ifndef RTM_H
#define RTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTM_ABI_VERSION 1

/* Status codes. */
#define RTM_OK 0
#define RTM_EINVAL (-1)     /* bad argument: null pointer, size, dimension      */
#define RTM_ECFL (-2)       /* max(v) dt / h >= sqrt(315 / (512 d)): unstable   */
#define RTM_ERANGE (-3)     /* a source or receiver lies outside the interior   */
#define RTM_EWORKSPACE (-4) /* workspace null or smaller than required          */
#define RTM_EHIP (-5)       /* a HIP runtime call or kernel launch failed       */
#define RTM_ENUMERIC (-6)   /* velocity non-finite, negative or all zero; or a  */
                            /* non-finite output under RTM_F_CHECK_FINITE       */

/* Operations, for rtm_workspace_bytes. */
#define RTM_OP_RBC_PAD 0 /* rtm_rbc_pad and rtm_pad_adjoint with v_cap <= 0 */
#define RTM_OP_MODEL 1   /* rtm_model_shot                                  */
#define RTM_OP_RTM 2     /* rtm_rtm_shot                                    */
#define RTM_OP_VJP 3     /* rtm_model_shot_vjp                              */
#define RTM_OP_STORAGE 4 /* rtm_storage_shot                                */

/* Flags for rtm_model_shot, rtm_rtm_shot and rtm_model_shot_vjp. */
#define RTM_F_SKIP_CHECK 0x1u /* skip the velocity range check            */
#define RTM_F_NO_REINJECT 0x2u /* rtm_rtm_shot: reconstruct with a zero right
                                  side, as Eq. (6) is written (the wavelet is
                                  then not removed while it is active) */
#define RTM_F_ACCUMULATE 0x4u  /* batch RTM: add each shot's image into its
                                  image buffer (shots may share one buffer:
                                  the stacking of Algorithm 3) */
#define RTM_F_GRAPH 0x8u       /* batch: capture the launch schedule in a
                                  hipGraph on the first run and replay it on
                                  later runs with the same workspace and
                                  stream (stream must not be NULL) */
#define RTM_F_PERSISTENT 0x20u  /* 2-D batch: each pass (forward, reverse) is
                                  one launch of a resident grid that walks
                                  every time step, each shot's step waiting
                                  only for that shot's previous step (per-
                                  shot progress counters); one strip per
                                  workgroup, one step per pass over a tile.
                                  rtm_batch_run then synchronises the
                                  stream at the end and returns RTM_EHIP if
                                  a bounded wait gave up (the grid was not
                                  resident).  Not with RTM_F_GRAPH. */
#define RTM_F_CHECK_FINITE 0x10u /* single-shot calls: after the run, check
                                  the outputs (traces, image, or velocity
                                  gradient) for NaN / Inf; synchronises the
                                  stream and returns RTM_ENUMERIC if found */

/* Grid descriptor; read during the call only. */
typedef struct rtm_grid {
    int32_t ndim; /* 2 or 3 */
    int32_t nb;   /* random-boundary width in cells, on every face, >= 0 */
    int64_t nx, ny, nz; /* interior extents (ny = 1 in 2-D) */
    double h;     /* grid spacing in metres, > 0 */
} rtm_grid_t;

/* Optional wavefield probe of rtm_rtm_shot: copies the reconstructed source
 * wavefield p^k and the receiver wavefield mu^k at step k = snap_k
 * (0 <= snap_k <= nt - 2) into dense padded device fields. */
typedef struct rtm_probe {
    int32_t snap_k;
    float *snap_p;  /* device [NZ][NY][NX] or NULL */
    float *snap_mu; /* device [NZ][NY][NX] or NULL */
} rtm_probe_t;

/* ABI version implemented by the loaded library (RTM_ABI_VERSION). */
int rtm_abi_version(void);

/* Message for the last failing call on this thread ("" if none).  The
 * string is owned by the library and valid until the next call. */
const char *rtm_last_error(void);

/* Launch shape of the 2-D propagation kernels, process-wide, for the
 * autotuner: `op` RTM_OP_MODEL selects the forward kernel, RTM_OP_RTM or
 * RTM_OP_VJP the reverse kernels; vec in {1, 2, 4} floats per lane (strips
 * of 64 * vec columns), zseg rows per tile, a multiple of 9 in [9, 4095]
 * (the march is unrolled by the 9-row register queue).  A job with too few
 * tiles to fill the GPU gets a narrower shape automatically, unless
 * rtm_set_tuning(RTM_TUNE_EXACT, 1, 0) was called (RTM_TUNE_EXACT, 0, 0
 * re-enables narrowing).  Results do not depend on the shape.  Not
 * synchronised with concurrent calls. */
#define RTM_TUNE_EXACT 0x100
int rtm_set_tuning(int op, int vec, int zseg);
/* Current launch shape for `op` (same selection as rtm_set_tuning);
 * op RTM_TUNE_EXACT returns the no-narrowing setting (0 or 1) in *vec and 0
 * in *zseg. */
int rtm_get_tuning(int op, int *vec, int *zseg);

/* Full 2-D launch shape: as rtm_set_tuning plus tx in {1, 2, 4}
 * wavefronts per workgroup, each on one of tx adjacent strips.  The strips
 * of a workgroup pass their inner end cells to each other through LDS
 * instead of reloading them from memory.  rtm_set_tuning keeps the current
 * tx. */
int rtm_set_tuning2d(int op, int vec, int tx, int zseg);
int rtm_get_tuning2d(int op, int *vec, int *tx, int *zseg);

/* Time steps per launch of the 2-D propagation, 1, 2 or 3.  With 2, one
 * launch advances two steps: each wavefront computes the first step on its
 * strip plus a 4-cell margin and the second on the strip's inner columns
 * (strips overlap by 8 columns), and the two new levels go to a second set
 * of field buffers, so the level pairs cross HBM once per two steps.  With
 * 3 the strips overlap by 16 columns, the middle level stays in registers
 * (modeling stores it on the receiver rows only) and the last two levels
 * are stored: the pairs cross HBM once per three steps.  RTM_OP_MODEL sets
 * it for every forward pass (modeling and the forward pass of RTM and VJP
 * jobs; storage RTM, which copies whole levels, takes 2 when 3 is set; a
 * job too small to fill the GPU takes 2 unless RTM_TUNE_EXACT is set),
 * RTM_OP_RTM for the imaging reverse pass and the gradient pass (which
 * takes at most 2; probed runs take one step per launch; the last nt mod S
 * steps are taken one at a time).  Results are bit-identical whatever the
 * setting.
 * Returns RTM_EINVAL for other values. */
int rtm_set_steps_per_launch(int op, int steps);
int rtm_get_steps_per_launch(int op, int *steps);

/* Launch shape of the 3-D kernels: vec floats per lane (x strips of
 * 64 * vec cells), ty in {4, 8, 16} wavefronts per workgroup (rows in y),
 * zseg planes per tile (a multiple of 9).  ty 16 (1024-thread workgroups)
 * takes vec 1 or 2 for RTM_OP_MODEL and vec 1 for RTM_OP_RTM / RTM_OP_VJP.
 * Same rules as rtm_set_tuning. */
int rtm_set_tuning3d(int op, int vec, int ty, int zseg);
int rtm_get_tuning3d(int op, int *vec, int *ty, int *zseg);

/* Numbering of the 3-D tiles, process-wide per operation (RTM_OP_MODEL: the
 * forward kernels; RTM_OP_RTM / RTM_OP_VJP: the reverse ones): z_inner 0
 * (default) numbers them z band by z band with the y tiles innermost,
 * z_inner 1 x strip by x strip with the z bands innermost.  Workgroups are
 * dealt to the XCDs in that order, so it decides which tiles share an L2;
 * results do not depend on it (every cell's arithmetic is the same).  The
 * faster order depends on the grid (the autotuner tries both).
 * rtm_set_tuning3d keeps it.  RTM_EINVAL for z_inner other than 0 or 1 or an
 * unknown op. */
int rtm_set_tile_order3d(int op, int z_inner);
int rtm_get_tile_order3d(int op, int *z_inner);

/* Bounded wait of RTM_F_PERSISTENT passes, process-wide: a workgroup that
 * waits longer than `ms` milliseconds for its shot's previous step gives
 * up, the pass ends and rtm_batch_run returns RTM_EHIP (default 4000 ms;
 * [0, 3.6e6]).  Lowering it forces that path, for tests of the failure
 * handling.  Not synchronised with concurrent calls. */
int rtm_set_persist_wait(double ms);
int rtm_get_persist_wait(double *ms);

/* Event timing of the time loops, for measurement.  While enabled, every
 * propagation call records a HIP event pair on its stream around each of
 * its time loops (no host synchronisation is added).  rtm_timing_read waits
 * for the recorded events, returns the summed loop times in milliseconds
 * and the number of kernel launches they cover, per loop kind:
 *   [0] forward with receiver sampling (rtm_model_shot),
 *   [1] forward without sampling (rtm_rtm_shot, rtm_model_shot_vjp,
 *       rtm_storage_shot, whose snapshot copies it includes),
 *   [2] reverse with imaging (rtm_rtm_shot: fused reconstruction and
 *       receiver wavefield; rtm_storage_shot: receiver wavefield alone),
 *   [3] fused reverse with the gradient (rtm_model_shot_vjp),
 * and clears the record.  ms and launches point to 4 elements each.
 * Loops of calls given a probe are not recorded. */
int rtm_timing_enable(int on);
int rtm_timing_read(double *ms, int64_t *launches);

/* Bytes of device workspace needed by `op` on `grid` with nrec receivers
 * and nt time steps (nrec, nt ignored for RTM_OP_RBC_PAD).  Writes *bytes. */
int rtm_workspace_bytes(const rtm_grid_t *grid, int op, int32_t nrec, int32_t nt,
                        size_t *bytes);

/* Random boundary padding (Sec. "Wavefield Reconstruction": velocities in
 * the boundary band are randomised so that boundary returns do not
 * correlate coherently; they must respect the stability limit).
 *   v_int  device [nz][ny][nx] interior velocities (m/s), > 0.
 *   v_pad  device [NZ][NY][NX] output: interior copied; a band cell j takes
 *          min(f_j * v_edge(j), v_cap) in FP32, where v_edge(j) is the
 *          interior velocity at j's coordinates clamped into the interior,
 *          f_j = fmaf(0.6f, u_j, 0.7f) is uniform in [0.7, 1.3), and u_j is
 *          the top 24 bits of SplitMix64 (Steele, Lea & Flood 2014) output
 *          number j + 1 of the stream seeded with `seed`, times 2^-24, j the
 *          padded linear index.  The result is a pure function of
 *          (v_int, seed, v_cap): bit-for-bit reproducible.
 *   v_cap  cap in m/s; v_cap <= 0 uses max(v_int), which needs `ws` of
 *          rtm_workspace_bytes(RTM_OP_RBC_PAD) bytes (else ws may be NULL). */
int rtm_rbc_pad(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap,
                float *v_pad, void *ws, size_t ws_bytes, void *stream);

/* Band options of the random boundary: the paper's setup (Sec. "Wavefield
 * Reconstruction", Eqs. (4)-(5); the models of the 2-D and 3-D tests put
 * no band above the surface). */
#define RTM_RBC_TAPER 0x1u        /* scale band velocities by c_i, see below */
#define RTM_RBC_FREE_SURFACE 0x2u /* zero velocity above the interior       */

typedef struct rtm_rbc_opts {
    uint64_t seed;
    float v_cap;         /* as in rtm_rbc_pad */
    uint32_t flags;      /* RTM_RBC_TAPER | RTM_RBC_FREE_SURFACE or 0 */
    double taper_alpha;  /* RTM_RBC_TAPER: weight in [0, 1] of Eq. (4) */
} rtm_rbc_opts_t;

/* rtm_rbc_pad with band options.  Let i in [1, nb] be a band cell's depth,
 * the largest per-axis distance from the interior (i = 1 touches it).
 *  - RTM_RBC_TAPER: the value is min(c_i * (f_j * v_edge), v_cap) (FP32
 *    products in that order) with c_i = a g(i) + (1 - a) h(i), a =
 *    taper_alpha, g(i) = (nb - i)/(nb - 1) (Eq. (4)) and h(i) =
 *    exp(-120 (i - 1)^2 / (nb - 1)^2) (Eq. (5)), evaluated in double and
 *    rounded once to FP32 (c_1 = 1; nb = 1 gives 1).  So h <= c_i <= g and
 *    the band slows to ~0 at the outer face.  Needs nb <= 256.
 *  - RTM_RBC_FREE_SURFACE: every cell above the interior (z < nb) gets
 *    v = 0.  D' = 0 there, so p stays zero: the pressure-release surface of
 *    Eq. (1)'s Dirichlet condition sits one row above the interior, as with
 *    the paper's half-stencil top pad.
 * Propagation calls accept zero velocities (and return a zero velocity
 * gradient there).  opts is read during the call; other arguments and
 * errors as in rtm_rbc_pad. */
int rtm_rbc_pad_ex(const rtm_grid_t *grid, const float *v_int, const rtm_rbc_opts_t *opts,
                   float *v_pad, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of rtm_rbc_pad_ex with respect to v_int: as rtm_pad_adjoint with
 * the factor c_i f_j (FP32 product) under RTM_RBC_TAPER; free-surface cells
 * contribute nothing. */
int rtm_pad_adjoint_ex(const rtm_grid_t *grid, const float *v_int, const rtm_rbc_opts_t *opts,
                       const float *grad_v_pad, float *grad_v_int, void *ws, size_t ws_bytes,
                       void *stream);

/* Adjoint of rtm_rbc_pad with respect to v_int, the random factors and
 * v_cap held fixed: grad_v_int[i] = grad_v_pad[i] + sum of f_j grad_v_pad[j]
 * over band cells j whose edge cell is i and whose value was not capped.
 *   grad_v_pad device [NZ][NY][NX]; grad_v_int device [nz][ny][nx] output.
 *   Deterministic (gather, no atomics).  ws as for rtm_rbc_pad. */
int rtm_pad_adjoint(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap,
                    const float *grad_v_pad, float *grad_v_int, void *ws, size_t ws_bytes,
                    void *stream);

/* Seismic modeling of one shot (Algorithm 1 / Algorithm 4): zero initial
 * state, nt steps of Eq. (1), recording at the receivers.
 *   v_pad    device [NZ][NY][NX] padded velocity (from rtm_rbc_pad).
 *   wavelet  device [nt].
 *   src      host float[3]; rec host float[nrec][3] (nrec >= 1).
 *   traces   device [nrec][nt + 1] output.
 *   p_last, p_prev  device [NZ][NY][NX] or NULL: the final states p^nt and
 *            p^(nt-1), the two panels reconstruction starts from.
 *   flags    RTM_F_SKIP_CHECK | RTM_F_CHECK_FINITE or 0. */
int rtm_model_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                   const float *wavelet, const float *src, int32_t nrec, const float *rec,
                   float *traces, float *p_last, float *p_prev, uint32_t flags, void *ws,
                   size_t ws_bytes, void *stream);

/* Reverse time migration of one shot with random boundaries and source
 * wavefield reconstruction (Algorithm 3 / Algorithm 6, Eqs. (2), (3), (6)).
 * Forward pass as rtm_model_shot keeping the last two panels in device
 * memory; reverse pass k = nt-1 .. 0 stepping, in one fused kernel per step,
 *  - the reconstructed source wavefield, re-injecting the wavelet so that
 *    the reversal is exact up to rounding (RTM_F_NO_REINJECT: Eq. (6) as
 *    written);
 *  - the receiver wavefield as the exact adjoint of the forward scheme,
 *    driven by `traces` (mu^k = 2mu^{k+1} - mu^{k+2} + (v dt)^2 (L_h mu^{k+1}
 *    + R^T g^k)), from mu^{nt+1} = mu^{nt+2} = 0;
 *  - the two integrals of Eq. (3), pairing p^k with mu^{k+1}:
 *    num += p^k mu^{k+1}, den += (p^k)^2 (FP32 accumulators).
 * Output: image = num / (den + eps_rel * max(den)) on the interior.
 *   traces   device [nrec][nt + 1] recorded data.
 *   image    device [nz][ny][nx] output; num, den likewise or NULL.
 *   eps_rel  stabiliser >= 0.  1e-3 is recommended: with much smaller values
 *            the ratio divides by illumination far below its peak, where the
 *            FP32 wavefields carry large relative errors (the image error
 *            grows roughly like 1e-9 / eps_rel).
 *   probe    NULL or a wavefield probe (see rtm_probe_t).
 *   flags    RTM_F_SKIP_CHECK | RTM_F_NO_REINJECT | RTM_F_CHECK_FINITE or 0.
 * The caller stacks images over shots (Algorithm 3, stacking step). */
int rtm_rtm_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                 const float *wavelet, const float *src, int32_t nrec, const float *rec,
                 const float *traces, float eps_rel, float *image, float *num, float *den,
                 const rtm_probe_t *probe, uint32_t flags, void *ws, size_t ws_bytes,
                 void *stream);

/* rtm_rtm_shot for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation with no workspace argument and no probe.
 * Its scratch is a fixed array of RTM_NOALLOC_SCRATCH_BYTES bytes inside the
 * library, one per GPU, held from the library's load until the process
 * ends; the call allocates no device memory.  A shot whose
 * rtm_workspace_bytes(RTM_OP_RTM) exceeds that size is refused with
 * RTM_EWORKSPACE before any work is queued (the 201 x 201 two-layer shot
 * with its 40-cell band and 1000 steps needs about 6.3 MiB; a 1201 x 300
 * window with a 40-cell band and 2000 steps about 36 MiB).  The array
 * keeps the last call's contents, and every field the run reads is cleared
 * first, so results do not depend on earlier calls.
 * All calls on one GPU share its array: calls that overlap in time on one
 * GPU (other streams or host threads) race and give wrong results; order
 * them.  Other arguments, flags and errors as in rtm_rtm_shot. */
#define RTM_NOALLOC_SCRATCH_BYTES (64u << 20)
int rtm_rtm_shot_noalloc(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                         const float *wavelet, const float *src, int32_t nrec, const float *rec,
                         const float *traces, float eps_rel, float *image, float *num, float *den,
                         uint32_t flags, void *stream);

/* Snapshot step of the stored source wavefield (Eq. (7)): the Nyquist
 * interval 1 / (2 (f_max - f_min)) of a source band [f_min, f_max] Hz, in
 * whole time steps of dt seconds, at least 1.  Host only.
 * RTM_EINVAL unless dt > 0, 0 <= f_min < f_max, all finite. */
int rtm_nyquist_stride(double dt, double f_max, double f_min, int32_t *stride);

/* Number of stored levels of rtm_storage_shot: the k in [0, nt - 1] with
 * k = phase (mod stride).  Host only.  RTM_EINVAL unless nt >= 1,
 * stride >= 1 and 0 <= phase < stride. */
int rtm_storage_count(int32_t nt, int32_t stride, int32_t phase, int64_t *count);

/* Reverse time migration of one shot with a stored source wavefield
 * (Algorithm 2, the paper's comparison method), the snapshots kept in
 * device memory instead of on disk and decimated in time as in Eq. (7).
 * Forward pass as in rtm_rtm_shot; after reaching each stored level p^k
 * (k in [0, nt - 1], k = phase mod stride) its interior is copied into
 * `snapshots`.  Reverse pass k = nt-1 .. 0: only the receiver wavefield
 * (the same scheme and arithmetic as rtm_rtm_shot's), and at every stored
 * level the sums of Eq. (3) with the stored p^k:
 *    num += p^k mu^{k+1},  den += (p^k)^2.
 * With stride 1 the sums are those of rtm_rtm_shot up to the rounding of
 * its reconstructed p; a larger stride sums over the stored levels only
 * (no interpolation between them).
 *   traces     device [nrec][nt + 1] recorded data.
 *   stride, phase  decimation (see rtm_storage_count; rtm_nyquist_stride
 *              gives the paper's stride).
 *   eps_rel, image, num, den  as in rtm_rtm_shot.
 *   snapshots  device, caller-owned, count * nz * ny * nx floats: level i
 *              of the count stored ones (k = phase + i stride) at offset
 *              i * nz * ny * nx, dense interior [nz][ny][nx].  Valid after
 *              the call (the stored source wavefield).
 *   snapshot_bytes  size of `snapshots`; RTM_EINVAL if smaller than needed.
 *   flags      RTM_F_SKIP_CHECK | RTM_F_CHECK_FINITE or 0.
 *   ws         rtm_workspace_bytes(RTM_OP_STORAGE) bytes. */
int rtm_storage_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                     const float *wavelet, const float *src, int32_t nrec, const float *rec,
                     const float *traces, int32_t stride, int32_t phase, float eps_rel,
                     float *image, float *num, float *den, float *snapshots,
                     size_t snapshot_bytes, uint32_t flags, void *ws, size_t ws_bytes,
                     void *stream);

/* Vector-Jacobian product of rtm_model_shot with respect to the padded
 * velocity: given dJ/dtraces, returns dJ/dv_pad = 2 G / (v^3 dt^2) with
 * G = sum_k mu^{k+1} (p^{k+1} - 2p^k + p^{k-1}), mu driven by grad_traces
 * as in rtm_rtm_shot and p reconstructed from the last two panels (no
 * wavefield storage).
 *   grad_traces  device [nrec][nt + 1].
 *   grad_v_pad   device [NZ][NY][NX] output.
 *   grad_wavelet device [nt] output or NULL: dJ/dw^n = <delta_s / h^d, mu^{n+1}>. */
int rtm_model_shot_vjp(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                       const float *wavelet, const float *src, int32_t nrec,
                       const float *rec, const float *grad_traces, float *grad_v_pad,
                       float *grad_wavelet, uint32_t flags, void *ws, size_t ws_bytes,
                       void *stream);

/* ---------------------------------------------------------------------
 * Batches: many shots, possibly of different grids (uneven apertures),
 * propagated together.  Every time step is one kernel launch covering all
 * tiles of all shots; shots given the same v_pad pointer and grid share one
 * scaled-velocity array.  All shots use the same dt and nt.
 * --------------------------------------------------------------------- */

/* One shot of a batch.  Device buffers must stay valid while the plan is
 * run; `rec` (host) is read by rtm_batch_plan only. */
typedef struct rtm_shot_desc {
    rtm_grid_t grid;          /* this shot's grid */
    const float *v_pad;       /* device [NZ][NY][NX] padded velocity */
    const float *wavelet;     /* device [nt] */
    float src[3];             /* source position (interior grid units) */
    int32_t nrec;             /* >= 1 */
    const float *rec;         /* host [nrec][3] */
    const float *traces_in;   /* device [nrec][nt + 1]: recorded data (RTM) or
                                 dJ/dtraces (VJP); unused for modeling */
    float *traces_out;        /* device [nrec][nt + 1]: modeling output */
    float *image;             /* device [nz][ny][nx]: RTM image, written or
                                 accumulated (RTM_F_ACCUMULATE) */
    float *grad_v_pad;        /* device [NZ][NY][NX]: VJP output */
} rtm_shot_desc_t;

typedef struct rtm_plan rtm_plan_t;

/* Validates the shots, builds their tiles and injection tables with the
 * current launch shapes, and returns an opaque plan (host memory only)
 * plus the workspace size its runs need.  op is RTM_OP_MODEL, RTM_OP_RTM
 * or RTM_OP_VJP; flags: RTM_F_SKIP_CHECK, RTM_F_NO_REINJECT (RTM),
 * RTM_F_ACCUMULATE (RTM), RTM_F_GRAPH, RTM_F_PERSISTENT (2-D).  eps_rel as
 * in rtm_rtm_shot. */
int rtm_batch_plan(int op, int32_t nshots, const rtm_shot_desc_t *shots, double dt, int32_t nt,
                   float eps_rel, uint32_t flags, rtm_plan_t **plan, size_t *ws_bytes);

/* Runs a plan on `stream` with a workspace of at least the planned size
 * (256-byte aligned).  Uploads the tables, checks velocities (one stream
 * synchronisation), then queues the propagation.  Results equal those of
 * the single-shot entry points bit for bit.  Runs of one plan must not
 * overlap in time. */
int rtm_batch_run(rtm_plan_t *plan, void *ws, size_t ws_bytes, void *stream);

/* Releases a plan (and its graph); NULL is allowed. */
int rtm_batch_free(rtm_plan_t *plan);

/* Shots of uneven aperture see windows of one wide 2-D model.  For
 * [nz][nx_global] device arrays and 0 <= x0, x0 + width <= nx_global:
 * rtm_window_extract copies columns [x0, x0 + width) into a dense
 * [nz][width] window; rtm_window_accumulate adds a window back into them
 * (the adjoint of the extraction).  Calls on one stream run in order, so
 * accumulating overlapping windows one after another is deterministic. */
int rtm_window_extract(int64_t nz, int64_t nx_global, int64_t x0, int64_t width, const float *global,
                       float *window, void *stream);
int rtm_window_accumulate(int64_t nz, int64_t nx_global, int64_t x0, int64_t width, const float *window,
                          float *global, void *stream);

/* Receiver subtraction and the L2 misfit of modeled traces: residual =
 * d - d_obs (device [n], may be NULL) and *J = 0.5 sum residual^2 written to
 * a device double.  The sum runs in a fixed order (per-block partials in
 * FP64, then one block over the partials): deterministic.  ws: device,
 * 256-byte aligned, rtm_misfit_ws_bytes bytes. */
int rtm_misfit_ws_bytes(size_t *bytes);
int rtm_l2_misfit(int64_t n, const float *d, const float *d_obs, float *residual, double *J, void *ws,
                  size_t ws_bytes, void *stream);

/* Streaming device-to-device copy of `bytes` bytes (16-byte loads and
 * stores, each read and written once), queued on `stream`: the measured
 * bandwidth reference for the propagation kernels' roofline (a plain
 * streaming kernel of known traffic, 2 * bytes per call).  src and dst are
 * device buffers that must not overlap; both addresses and `bytes` must be
 * multiples of 16 (RTM_EINVAL otherwise).  blocks_per_cu in [1, 64] sets the
 * grid: 256 workgroups of 256 threads per unit, each striding over the
 * buffer. */
int rtm_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RTM_H */
