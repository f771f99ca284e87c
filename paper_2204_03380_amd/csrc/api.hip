// Host runtime of librtm: argument validation, acquisition tables,
// workspace carving and the launch sequences behind the C ABI of
// include/rtm.h.  Every device buffer comes from the caller.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.h"
#include "rtm.h"

namespace rtm {
// prop2d.hip
hipError_t launch_fwd2d(int vec, int tx, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st);
hipError_t launch_rev2d(int vec, int tx, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles,
                        int nslots, const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj,
                        hipStream_t st);
hipError_t launch_fwd2d_t2(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                           hipStream_t st);
hipError_t launch_rev2d_t2(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st);
hipError_t launch_fwd2d_t3(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                           hipStream_t st);
hipError_t launch_rev2d_t3(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, int k, int reinject, hipStream_t st);
hipError_t launch_fwd2d_persist(int vec, const ShotDev *shots, const Tile2D *tiles, const PItem *items, int nitems,
                                const int *shot_items, const InjEnt *ents, const Contrib *cont,
                                const SampleTask *stasks, int n0, int nsteps, unsigned *cnt, unsigned *status,
                                double wait_ms, hipStream_t st);
hipError_t launch_rev2d_persist(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, const PItem *items,
                                int nitems, const int *shot_items, const InjEnt *ents, const Contrib *cont, int k0,
                                int nsteps, int reinject, float *wadj, unsigned *cnt, unsigned *status,
                                double wait_ms, hipStream_t st);
hipError_t launch_recv2d(int vec, int tx, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                         const InjEnt *ents, const Contrib *cont, int k, const float *snap, hipStream_t st);
// prop3d.hip
hipError_t launch_fwd3d(int vec, int ty, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st);
hipError_t launch_rev3d(int vec, int ty, bool grad, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st);
hipError_t launch_recv3d(int vec, int ty, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                         const InjEnt *ents, const Contrib *cont, int k, const float *snap, hipStream_t st);
// aux.hip
hipError_t launch_vrange(const float *v, int64_t n, unsigned *maxmin2, hipStream_t st);
hipError_t launch_vmax(const float *v, int64_t n, unsigned *out, hipStream_t st);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t units, int blocks_per_cu, hipStream_t st);
hipError_t launch_rbc_pad(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int, uint64_t seed,
                          float v_cap, const unsigned *cap_bits, const BandOpts &o, float *v_pad, hipStream_t st);
hipError_t launch_pad_adjoint(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int,
                              uint64_t seed, float v_cap, const unsigned *cap_bits, const BandOpts &o,
                              const float *g_pad, float *g_int, hipStream_t st);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_build_dp(const Layout &L, const float *v_pad, float dt_over_h, float *Dp, hipStream_t st);
hipError_t launch_unpack(const Layout &L, const float *f, float *out, hipStream_t st);
hipError_t launch_transpose(const float *in, float *out, int64_t R, int64_t C, hipStream_t st);
hipError_t launch_inj_set(const ShotDev *shots, const InjEnt *ents, int ebeg, int eend, const Contrib *cont, int step,
                          hipStream_t st);
hipError_t launch_sample(const ShotDev *shots, const SampleTask *stasks, int ntask, int n, int slot, hipStream_t st);
hipError_t launch_image(const ShotDev *shots, int shot, int64_t ninterior, unsigned *dmax_bits, float eps_rel,
                        float *image, int accumulate, float *num, float *den, hipStream_t st);
hipError_t launch_grad(const ShotDev *shots, int shot, int64_t npad, const float *v_pad, float dt, float *grad,
                       hipStream_t st);
hipError_t launch_snap_store(const ShotDev *shots, int shot, int lev, int64_t ninterior, float *out, hipStream_t st);
hipError_t launch_nonfinite(const float *x, int64_t n, unsigned *flag, hipStream_t st);
hipError_t launch_wadj(const float *parts, int nt, float scale, float *out, hipStream_t st);
size_t misfit_ws_bytes();
hipError_t launch_misfit(const float *d, const float *dobs, float *r, int64_t n, void *ws, double *J, hipStream_t st);
hipError_t launch_window(float *global, const float *win_in, float *win_out, int64_t nz, int64_t nxg, int64_t x0,
                         int64_t w, int mode, hipStream_t st);
}  // namespace rtm

using namespace rtm;

namespace {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

thread_local std::string t_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

}  // namespace

// Error state shared with the other sources of the library.
namespace rtm {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
void clear_error() { t_err.clear(); }
}  // namespace rtm

namespace {

#define RTM_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(RTM_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Tuning: strip width (VEC floats per lane) and rows per tile.
// ---------------------------------------------------------------------------

struct Tune {
    int vec;
    int zseg;
    int ty;  // 3-D: wavefronts (y rows) per workgroup
    int tx;  // 2-D: wavefronts (adjacent strips) per workgroup
    int steps = 1;  // 2-D: time steps per launch (1, 2 or 3)
    int zin = 0;    // 3-D: tiles numbered with z innermost (else y innermost)
};

// 2-D shapes: ((steps - 1) << 28) | (tx << 24) | (vec << 16) | zseg;
// defaults from sweeps over 48 shots of the 2301 x 751 folded grid: three
// steps per launch at vec 2, 108-row tiles (reverse 412 us per step, RTM
// forward 153; two steps at vec 4 took 584 and 212, three at vec 4 545 and
// 201).  Modeling, which takes two steps per launch, then runs at vec 2
// (232 us per step against 213 at vec 4).
std::atomic<int> g_tune2d_fwd{(2 << 28) | (1 << 24) | (2 << 16) | 108};
std::atomic<int> g_tune2d_rev{(2 << 28) | (1 << 24) | (2 << 16) | 108};
std::atomic<int> g_tune_exact{0};  // 1: never narrow the configured shapes
std::atomic<double> g_persist_wait_ms{4000.0};  // bounded wait of persistent passes

// 3-D shapes: (vec << 24) | (ty << 16) | (z_inner << 15) | zseg; defaults from a sweep on
// the 612 x 612 x 356 padded layered-salt grid (us per step: forward 556 at
// vec 1, 4 rows, 18 planes against 575 at vec 2, 8 rows; reverse 1353).
std::atomic<int> g_tune3d_fwd{(1 << 24) | (4 << 16) | 18};
std::atomic<int> g_tune3d_rev{(1 << 24) | (4 << 16) | 18};

Tune get_tune(int which, int ndim)
{
    if (ndim == 3) {
        int v = (which == 0 ? g_tune3d_fwd : g_tune3d_rev).load();
        Tune t{v >> 24, v & 0x7fff, (v >> 16) & 0xff, 1};
        t.zin = (v >> 15) & 1;
        return t;
    }
    int v = (which == 0 ? g_tune2d_fwd : g_tune2d_rev).load();
    return Tune{(v >> 16) & 0xff, v & 0xffff, 1, (v >> 24) & 0xf, ((v >> 28) & 0x3) + 1};
}

constexpr int kMinZseg = kZUnroll;

// ---------------------------------------------------------------------------
// Optional event timing of the time loops (measurement only).
// ---------------------------------------------------------------------------

enum LoopKind { kLoopModelFwd = 0, kLoopRtmFwd = 1, kLoopRevImage = 2, kLoopRevGrad = 3, kLoopKinds = 4 };

struct PendingTiming {
    hipEvent_t start, stop;
    int kind;
    int64_t launches;
};

std::atomic<int> g_timing_on{0};
std::mutex g_timing_mu;
std::vector<PendingTiming> g_timing_pending;

// Records an event pair around [begin, end) of a loop on `st`; the pair is
// resolved later by rtm_timing_read, so no host synchronisation is added.
// A roctx range over one pass of a job's launch sequence (host time of the
// enqueues; shown by rocprofv3 --marker-trace, a no-op otherwise).
struct PassRange {
    explicit PassRange(const char *name) { roctxRangePushA(name); }
    ~PassRange() { roctxRangePop(); }
    PassRange(const PassRange &) = delete;
    PassRange &operator=(const PassRange &) = delete;
};

struct LoopTimer {
    hipEvent_t a = nullptr, b = nullptr;
    int kind;
    int64_t launches;
    hipStream_t st;
    LoopTimer(int k, int64_t n, hipStream_t s, bool enable = true) : kind(k), launches(n), st(s)
    {
        if (!enable || !g_timing_on.load()) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    void finish()
    {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_timing_mu);
        g_timing_pending.push_back(PendingTiming{a, b, kind, launches});
        a = b = nullptr;
    }
    ~LoopTimer()
    {
        // Loop abandoned on an error path: drop its events.
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// ---------------------------------------------------------------------------
// Grids and point operators
// ---------------------------------------------------------------------------

struct GridInfo {
    int ndim, nb;
    int64_t nx, ny, nz;
    int NX, NY, NZ;
    double h;
    Layout L;
};

int grid_info(const rtm_grid_t *g, GridInfo *gi)
{
    if (!g) return fail(RTM_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(RTM_EINVAL, "ndim must be 2 or 3 (got %d)", (int)g->ndim);
    if (g->nb < 0) return fail(RTM_EINVAL, "nb must be >= 0");
    int64_t ny = g->ndim == 3 ? g->ny : 1;
    if (g->nx < 1 || g->nz < 1 || ny < 1) return fail(RTM_EINVAL, "interior extents must be >= 1");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(RTM_EINVAL, "h must be positive and finite");
    int64_t NX = g->nx + 2 * (int64_t)g->nb, NZ = g->nz + 2 * (int64_t)g->nb;
    int64_t NY = g->ndim == 3 ? ny + 2 * (int64_t)g->nb : 1;
    if (NX > (1 << 28) || NY > (1 << 28) || NZ > (1 << 28)) return fail(RTM_EINVAL, "grid too large");
    gi->ndim = g->ndim;
    gi->nb = g->nb;
    gi->nx = g->nx;
    gi->ny = ny;
    gi->nz = g->nz;
    gi->NX = (int)NX;
    gi->NY = (int)NY;
    gi->NZ = (int)NZ;
    gi->h = g->h;
    gi->L = make_layout(g->ndim, (int)NX, (int)NY, (int)NZ);
    if (gi->L.total >= ((int64_t)1 << 31)) return fail(RTM_EINVAL, "field of %lld floats exceeds 2^31", (long long)gi->L.total);
    return RTM_OK;
}

struct PointOp {
    int n;
    int z[kMaxNodes], y[kMaxNodes], x[kMaxNodes];
    double w[kMaxNodes];
};

// Multilinear interpolation nodes (padded coordinates) and weights of an
// interior position; zero weights are dropped.
bool make_point(const GridInfo &g, const float *pos, PointOp *P)
{
    double q[3] = {pos[0], g.ndim == 3 ? pos[1] : 0.0, pos[2]};
    int64_t n[3] = {g.nx, g.ny, g.nz};
    int64_t i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        if (!(q[a] >= 0.0 && q[a] <= (double)(n[a] - 1))) return false;
        i0[a] = (int64_t)std::floor(q[a]);
        fr[a] = q[a] - (double)i0[a];
    }
    P->n = 0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double w = (cx ? fr[0] : 1 - fr[0]) * (cy ? fr[1] : 1 - fr[1]) * (cz ? fr[2] : 1 - fr[2]);
                if (w == 0.0) continue;
                P->x[P->n] = (int)(i0[0] + cx + g.nb);
                P->y[P->n] = g.ndim == 3 ? (int)(i0[1] + cy + g.nb) : 0;
                P->z[P->n] = (int)(i0[2] + cz + g.nb);
                P->w[P->n] = w;
                P->n++;
            }
    return true;
}

// ---------------------------------------------------------------------------
// Jobs: one or many shots propagated together.  Every time step is one
// kernel launch covering all tiles of all shots; shots with the same padded
// model and grid share their D' array.
// ---------------------------------------------------------------------------

struct ShotIn {
    GridInfo g;
    const float *v_pad = nullptr;
    const float *wavelet = nullptr;
    float src[3] = {0, 0, 0};
    int nrec = 0;
    std::vector<float> rec;             // [nrec][3]
    const float *traces_in = nullptr;   // RTM data / VJP upstream gradient, [nrec][nt + 1]
    float *traces_out = nullptr;        // modeling output, [nrec][nt + 1]
    float *image = nullptr, *num = nullptr, *den = nullptr;  // RTM outputs (interior)
    float *grad_v_pad = nullptr, *grad_wavelet = nullptr;    // VJP outputs
    float *p_last = nullptr, *p_prev = nullptr;              // modeling: final panels
    float *snaps = nullptr;             // storage RTM: stored interior levels
    int stride = 1, phase = 0;          // storage RTM: levels k = phase (mod stride)
};

// Tiles and injection entries of one launch shape.  ents holds all source
// entries of all shots, then all receiver entries (when present).
struct Tiling {
    Tune tune{1, 18, 1, 1, 1};
    int ndim = 2;
    int steps = 1;  // 2-D: time steps per launch of the tiles (> 1: overlapping strips)
    std::vector<Tile2D> tiles;   // 2-D jobs
    std::vector<Tile3D> tiles3;  // 3-D jobs
    std::vector<InjEnt> ents;
    std::vector<Contrib> cont;
    int nsrc_ent = 0, nrec_ent = 0, nslots = 0;
    int count() const { return ndim == 3 ? (int)tiles3.size() : (int)tiles.size(); }
};

struct Counts {
    int64_t tiles_f = 0, ents_f = 0, cont_f = 0;  // forward tiling
    int64_t tiles_r = 0, ents_r = 0, cont_r = 0;  // reverse tiling
    int64_t tiles_f2 = 0, ents_f2 = 0, cont_f2 = 0;  // multi-step tilings (2-D)
    int64_t tiles_r2 = 0, ents_r2 = 0, cont_r2 = 0;
    int64_t stasks = 0, rnode = 0;
    int64_t pitems_f = 0, pitems_r = 0;  // persistent passes: work items
};

// Byte offsets of every device buffer inside the workspace.
struct WsLayout {
    size_t scal = 0, shots = 0, tiles_f = 0, ents_f = 0, cont_f = 0, tiles_r = 0, ents_r = 0, cont_r = 0;
    size_t tiles_f2 = 0, ents_f2 = 0, cont_f2 = 0, tiles_r2 = 0, ents_r2 = 0, cont_r2 = 0;
    size_t stasks = 0, rnode = 0, rw = 0;
    size_t pitems_f = 0, pitems_r = 0, pnum = 0, pcnt = 0;  // persistent passes
    std::vector<size_t> dp;                  // per D' slot
    std::vector<std::array<size_t, 8>> fld;  // per shot
    std::vector<size_t> acc0, acc1, trint, wadj;
    size_t bytes = 0;
};

struct Job {
    int op = RTM_OP_MODEL;
    int nt = 0;
    double dt = 0.0;
    float eps = 1e-3f;
    uint32_t flags = 0;
    std::vector<ShotIn> shots;
    Tiling fw, rv;    // rv unused for modeling
    Tiling fw2, rv2;  // multi-step tilings (2-D, when the shape asks for two or three steps per launch)
    std::vector<SampleTask> stasks;
    std::vector<int> rnode;
    std::vector<float> rw;
    std::vector<int64_t> rbase;      // per shot: offset of its receivers in rnode / rw (in receivers)
    std::vector<std::array<int, 2>> srows;  // per shot: padded rows [lo, hi) holding receiver nodes
    std::vector<int> dslot;          // per shot: D' slot
    std::vector<int> slot_shot;      // per slot: first shot using it
    // persistent passes (RTM_F_PERSISTENT): work items and per-shot item
    // counts of the forward and reverse passes
    std::vector<PItem> pitems_f, pitems_r;
    std::vector<int> pnum;           // [0, nsh): forward, [nsh, 2 nsh): reverse
    WsLayout ws;
    // hipGraph of the launch schedule (plans with RTM_F_GRAPH)
    hipGraphExec_t gexec = nullptr;
    void *g_ws = nullptr;
    hipStream_t g_st = nullptr;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Field buffers per shot: p (2 levels) and mu (2 levels); 2-D jobs keep a
// second set for the multi-step kernels, so that the workspace size does not
// depend on the launch shape.  2-D modeling keeps, in the mu slot 2 of each
// set, the middle level that three-step launches store on the receiver rows.
int per_set(int op, int ndim) { return op == RTM_OP_MODEL ? (ndim == 2 ? 3 : 2) : 4; }
int nfields(int op, int ndim) { return per_set(op, ndim) * (ndim == 2 ? 2 : 1); }
int nfields(const Job &J) { return nfields(J.op, J.shots.empty() ? 3 : J.shots[0].g.ndim); }
// Ops with the imaging sums num (acc0) and den (acc1).
bool has_den(int op) { return op == RTM_OP_RTM || op == RTM_OP_STORAGE; }

constexpr size_t kTileBytes = sizeof(Tile2D) > sizeof(Tile3D) ? sizeof(Tile2D) : sizeof(Tile3D);

WsLayout make_ws_layout(const Job &J, const Counts &c)
{
    WsLayout w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align256(off);
        size_t o = off;
        off += bytes;
        return o;
    };
    const int nsh = (int)J.shots.size();
    const int nslot = (int)J.slot_shot.size();
    w.scal = take(sizeof(unsigned) * (64 + 2 * (size_t)nslot + (size_t)nsh));
    w.shots = take(sizeof(ShotDev) * 2 * nsh);  // two copies: field sets in either order
    w.tiles_f = take(kTileBytes * c.tiles_f);
    w.ents_f = take(sizeof(InjEnt) * c.ents_f);
    w.cont_f = take(sizeof(Contrib) * c.cont_f);
    w.tiles_r = take(kTileBytes * c.tiles_r);
    w.ents_r = take(sizeof(InjEnt) * c.ents_r);
    w.cont_r = take(sizeof(Contrib) * c.cont_r);
    w.tiles_f2 = take(kTileBytes * c.tiles_f2);
    w.ents_f2 = take(sizeof(InjEnt) * c.ents_f2);
    w.cont_f2 = take(sizeof(Contrib) * c.cont_f2);
    w.tiles_r2 = take(kTileBytes * c.tiles_r2);
    w.ents_r2 = take(sizeof(InjEnt) * c.ents_r2);
    w.cont_r2 = take(sizeof(Contrib) * c.cont_r2);
    w.stasks = take(sizeof(SampleTask) * c.stasks);
    w.rnode = take(sizeof(int) * c.rnode * kMaxNodes);
    w.rw = take(sizeof(float) * c.rnode * kMaxNodes);
    if (c.pitems_f > 0) {
        w.pitems_f = take(sizeof(PItem) * c.pitems_f);
        w.pitems_r = take(sizeof(PItem) * std::max<int64_t>(c.pitems_r, 1));
        w.pnum = take(sizeof(int) * 2 * (size_t)nsh);
        w.pcnt = take(sizeof(unsigned) * ((size_t)nsh + 1));  // per-shot counters, then the status word
    }
    for (int d = 0; d < nslot; ++d) w.dp.push_back(take(sizeof(float) * J.shots[J.slot_shot[d]].g.L.total));
    const int nf = nfields(J);
    for (int i = 0; i < nsh; ++i) {
        const ShotIn &S = J.shots[i];
        const int64_t F = S.g.L.total;
        // fields 0..3: first set (p, p, mu, mu), 4..7: second set; a
        // modeling job has the two p levels of each set (and in 2-D the
        // middle-level slot 2)
        std::array<size_t, 8> f{0, 0, 0, 0, 0, 0, 0, 0};
        const int per = per_set(J.op, S.g.ndim);  // fields per set
        for (int k = 0; k < nf; ++k) f[(k / per) * 4 + k % per] = take(sizeof(float) * F);
        w.fld.push_back(f);
        w.acc0.push_back(J.op == RTM_OP_MODEL ? 0 : take(sizeof(float) * F));
        w.acc1.push_back(has_den(J.op) ? take(sizeof(float) * F) : 0);
        w.trint.push_back(take(sizeof(float) * (size_t)(J.nt + 1) * S.nrec));
        w.wadj.push_back(J.op == RTM_OP_VJP ? take(sizeof(float) * (size_t)J.nt * kMaxNodes) : 0);
    }
    w.bytes = align256(off);
    return w;
}

int max_tiles(const GridInfo &g)
{
    const int64_t ny = g.ndim == 3 ? (g.NY + 3) / 4 : 1;
    return (int)(((int64_t)(g.NX + 63) / 64) * ny * (g.L.NZr / kMinZseg));
}

struct RawEnt {
    int tile, z, y, x;
    std::vector<Contrib> c;
    int slot, shot;
};

// Builds the tiles and injection entries of every shot for one launch shape.
int build_tiling(Job &J, Tiling &T, bool with_receivers)
{
    T.tiles.clear();
    T.tiles3.clear();
    T.ents.clear();
    T.cont.clear();
    std::vector<RawEnt> se, re;
    // 2-D: one tile is TX adjacent strips (one workgroup); 3-D: one strip.
    // 2-D tiles of S > 1 steps per launch: strips of 64 vec columns starting
    // at j W - 4 (S - 1) that own W = 64 vec - 8 (S - 1) columns each
    // (neighbours overlap by 8 (S - 1)).
    const bool two = T.ndim == 2 && T.steps > 1;
    const int off = two ? 4 * (T.steps - 1) : 0;
    const int span = 64 * T.tune.vec;
    const int strip = two ? span - 2 * off : span * (T.ndim == 2 ? T.tune.tx : 1);
    const int ty = T.ndim == 3 ? T.tune.ty : 1;
    for (int s = 0; s < (int)J.shots.size(); ++s) {
        const ShotIn &S = J.shots[s];
        const GridInfo &g = S.g;
        const int NZr = g.L.NZr;
        const int ns = (g.NX + strip - 1) / strip;
        const int nys = T.ndim == 3 ? (g.NY + ty - 1) / ty : 1;
        const int nzs = (NZr + T.tune.zseg - 1) / T.tune.zseg;
        const int tbase = T.count();
        // Tiles are numbered band by band in z, strip by strip within a band
        // and (3-D) y tile by y tile within a strip, so that the workgroups
        // that share lines run back to back on one XCD: adjacent 2-D strips
        // share their strip-end columns (measured 3-7 % faster than strip by
        // strip), adjacent 3-D y tiles the 4-row halos above and below.  A
        // 3-D tuning may number them z innermost instead (x strip, then y
        // tile, then z band), which some grids prefer (the better order
        // depends on the grid: measured, not derived).
        const bool zin = T.ndim == 3 && T.tune.zin;
        const int nA = zin ? ns : nzs, nB = zin ? nys : ns, nC = zin ? nzs : nys;
        for (int ia = 0; ia < nA; ++ia)
            for (int ib = 0; ib < nB; ++ib)
                for (int ic = 0; ic < nC; ++ic) {
                    const int zs = zin ? ic : ia, xs = zin ? ia : ib, ys = zin ? ib : ic;
                    const int z0 = zs * T.tune.zseg, z1 = std::min(z0 + T.tune.zseg, NZr);
                    if (T.ndim == 3) {
                        Tile3D t{};
                        t.shot = s;
                        t.x0 = xs * strip;
                        t.y0 = ys * ty;
                        t.z0 = z0;
                        t.z1 = z1;
                        T.tiles3.push_back(t);
                    } else {
                        Tile2D t{};
                        t.shot = s;
                        t.x0 = xs * strip - off;
                        t.z0 = z0;
                        t.z1 = z1;
                        T.tiles.push_back(t);
                    }
                }
        // (2-D multi-step: x is an owned column)
        auto tile_of = [&](int z, int y, int x) {
            if (zin) return tbase + ((x / strip) * nys + y / ty) * nzs + z / T.tune.zseg;
            return tbase + ((z / T.tune.zseg) * ns + x / strip) * nys + (T.ndim == 3 ? y / ty : 0);
        };
        PointOp sp;
        if (!make_point(g, S.src, &sp))
            return fail(RTM_ERANGE, "shot %d: source (%g, %g, %g) outside the interior", s, S.src[0], S.src[1],
                        S.src[2]);
        const double hd = std::pow(g.h, g.ndim);
        const double h2 = g.h * g.h;
        for (int q = 0; q < sp.n; ++q) {
            RawEnt e{tile_of(sp.z[q], sp.y[q], sp.x[q]), sp.z[q], sp.y[q], sp.x[q], {}, q, s};
            // D (B w) = D' (h^2 W / h^d) w with D' = (v dt / h)^2.
            e.c.push_back(Contrib{0, (float)(sp.w[q] * h2 / hd)});
            se.push_back(e);
        }
        if (!with_receivers) continue;
        std::map<std::tuple<int, int, int>, size_t> node_of;
        for (int r = 0; r < S.nrec; ++r) {
            PointOp rp;
            if (!make_point(g, &S.rec[3 * (size_t)r], &rp))
                return fail(RTM_ERANGE, "shot %d: receiver %d outside the interior", s, r);
            for (int q = 0; q < rp.n; ++q) {
                auto key = std::make_tuple(rp.z[q], rp.y[q], rp.x[q]);
                auto it = node_of.find(key);
                if (it == node_of.end()) {
                    it = node_of.emplace(key, re.size()).first;
                    re.push_back(RawEnt{tile_of(rp.z[q], rp.y[q], rp.x[q]), rp.z[q], rp.y[q], rp.x[q], {}, 0, s});
                }
                // D R^T g = D' h^2 W g.
                re[it->second].c.push_back(Contrib{r, (float)(rp.w[q] * h2)});
            }
        }
    }
    // Multi-step tiles also list, per tile, every node inside its strip and
    // rows [z0 - 4 (S - 1), z1 + 4 (S - 1)), where the first step is
    // computed; three-step tiles also those of rows [z0 - 4, z1 + 4), where
    // the second is.
    std::vector<RawEnt> se1, re1, se2, re2;
    if (two) {
        auto widen = [&](const std::vector<RawEnt> &v, std::vector<RawEnt> &out, int ext) {
            for (const RawEnt &e : v) {
                const ShotIn &S = J.shots[e.shot];
                const int NZr = S.g.L.NZr;
                const int ns = (S.g.NX + strip - 1) / strip;
                const int nzs = (NZr + T.tune.zseg - 1) / T.tune.zseg;
                int tb = 0;  // first tile of the shot
                for (int q = 0; q < e.shot; ++q) {
                    const ShotIn &o = J.shots[q];
                    tb += ((o.g.NX + strip - 1) / strip) * ((o.g.L.NZr + T.tune.zseg - 1) / T.tune.zseg);
                }
                // ext <= 8 < zseg and 2 off < strip: the node lies in z tiles
                // zc - 1 .. zc + 1 and strips jc - 1 .. jc at most
                const int jc = (e.x + off) / strip, zc = e.z / T.tune.zseg;
                for (int zs = std::max(0, zc - 1); zs <= std::min(nzs - 1, zc + 1); ++zs)
                    for (int j = std::max(0, jc - 2); j <= std::min(ns - 1, jc + 1); ++j) {
                        const int x0 = j * strip - off;
                        const int z0 = zs * T.tune.zseg, z1 = std::min(z0 + T.tune.zseg, NZr);
                        if (e.x >= x0 && e.x < x0 + span && e.z >= z0 - ext && e.z < z1 + ext) {
                            RawEnt w = e;
                            w.tile = tb + zs * ns + j;
                            out.push_back(w);
                        }
                    }
            }
        };
        widen(se, se1, off);
        widen(re, re1, off);
        if (T.steps == 3) {
            widen(se, se2, 4);
            widen(re, re2, 4);
        }
    }
    auto order = [](const RawEnt &a, const RawEnt &b) {
        return std::tie(a.tile, a.z, a.y, a.x) < std::tie(b.tile, b.z, b.y, b.x);
    };
    std::sort(se.begin(), se.end(), order);
    std::sort(re.begin(), re.end(), order);
    std::sort(se1.begin(), se1.end(), order);
    std::sort(re1.begin(), re1.end(), order);
    std::sort(se2.begin(), se2.end(), order);
    std::sort(re2.begin(), re2.end(), order);
    for (auto &t : T.tiles)
        t.sbeg = t.send = t.rbeg = t.rend = t.s1beg = t.s1end = t.r1beg = t.r1end = t.s2beg = t.s2end = t.r2beg =
            t.r2end = 0;
    for (auto &t : T.tiles3) t.sbeg = t.send = t.rbeg = t.rend = 0;
    // kind: 0 source, 1 receivers, 2 source (first step), 3 receivers (first
    // step), 4 source (second step), 5 receivers (second step)
    auto emit = [&](std::vector<RawEnt> &v, int kind) {
        for (auto &e : v) {
            InjEnt E{e.z, e.y, e.x, (int)T.cont.size(), 0, e.slot, e.shot, 0};
            for (auto &c : e.c) T.cont.push_back(c);
            E.cend = (int)T.cont.size();
            const int idx = (int)T.ents.size();
            T.ents.push_back(E);
            int *b, *n;
            if (T.ndim == 3) {
                Tile3D &t = T.tiles3[e.tile];
                b = kind == 0 ? &t.sbeg : &t.rbeg;
                n = kind == 0 ? &t.send : &t.rend;
            } else {
                Tile2D &t = T.tiles[e.tile];
                int *bs[6] = {&t.sbeg, &t.rbeg, &t.s1beg, &t.r1beg, &t.s2beg, &t.r2beg};
                int *ns_[6] = {&t.send, &t.rend, &t.s1end, &t.r1end, &t.s2end, &t.r2end};
                b = bs[kind];
                n = ns_[kind];
            }
            if (*n == *b) *b = idx;
            *n = idx + 1;
        }
    };
    emit(se, 0);
    T.nsrc_ent = (int)se.size();
    emit(re, 1);
    T.nrec_ent = (int)re.size();
    emit(se1, 2);
    emit(re1, 3);
    emit(se2, 4);
    emit(re2, 5);
    T.nslots = (T.count() + kNumXcd - 1) / kNumXcd * kNumXcd;
    return RTM_OK;
}

// Wavefronts a launch shape gives a job.
int64_t count_tiles(const Job &J, Tune t)
{
    int64_t n = 0;
    for (const ShotIn &S : J.shots) {
        const int64_t ny = S.g.ndim == 3 ? (S.g.NY + t.ty - 1) / t.ty * t.ty : 1;  // wavefronts per column
        const int64_t wx = S.g.ndim == 2 ? t.tx : 1;                                   // wavefronts per strip group
        n += (int64_t)((S.g.NX + 64 * t.vec * wx - 1) / (64 * t.vec * wx)) * wx * ny *
             ((S.g.L.NZr + t.zseg - 1) / t.zseg);
    }
    return n;
}

// The configured shape is meant for large batches; a small job (a single
// shot of a modest grid) would leave most of the 256 CUs idle, so the shape
// is narrowed (fewer rows per tile first, then fewer floats per lane) until
// the job has at least kMinWaves wavefronts or the smallest shape is
// reached.  Results do not depend on the shape.
//
// Three steps per launch keep their shape down to kT3Mid wavefronts, take
// half-height tiles down to kT3Small, and below that (one or two shots of a
// survey grid, latency-bound) give way to two steps and the narrowing
// above.  Measured per shot on 2301 x 751 batches (modeling + RTM): 2 shots
// 26-28 us per step with two steps against 33+ with three; 4 and 8 shots
// 26 and 18 us with three steps and half-height tiles against 27-29 and
// 24-31 otherwise; 16 shots and more best at the configured shape.
constexpr int64_t kMinWaves = 256 * 16;
constexpr int64_t kT3Mid = 2048, kT3Small = 600;

Tune fit_tune(const Job &J, Tune t)
{
    if (g_tune_exact.load()) return t;
    if (t.steps > 2) {
        const int64_t n = count_tiles(J, t);
        if (n >= kT3Mid) return t;
        if (n >= kT3Small) {
            if (t.zseg >= 2 * kMinZseg) t.zseg = std::max(kMinZseg, t.zseg / 2 / kZUnroll * kZUnroll);
            return t;
        }
        t.steps = 2;
    }
    while (count_tiles(J, t) < kMinWaves) {
        if (t.zseg > kMinZseg) t.zseg = std::max(kMinZseg, t.zseg / 2 / kZUnroll * kZUnroll);
        else if (t.ty > 4) t.ty = 4;
        else if (t.vec > 1) t.vec /= 2;
        else break;
    }
    return t;
}

// Receiver sampling tables, D' sharing and tilings of a job.
int build_job_tables(Job &J)
{
    J.stasks.clear();
    J.rnode.clear();
    J.rw.clear();
    J.rbase.clear();
    J.srows.clear();
    J.dslot.clear();
    J.slot_shot.clear();
    int64_t base = 0;
    for (int s = 0; s < (int)J.shots.size(); ++s) {
        const ShotIn &S = J.shots[s];
        J.rbase.push_back(base);
        std::array<int, 2> rows{1 << 30, 0};
        for (int r = 0; r < S.nrec; ++r) {
            PointOp rp;
            if (!make_point(S.g, &S.rec[3 * (size_t)r], &rp))
                return fail(RTM_ERANGE, "shot %d: receiver %d (%g, %g, %g) outside the interior", s, r,
                            S.rec[3 * r], S.rec[3 * r + 1], S.rec[3 * r + 2]);
            for (int q = 0; q < kMaxNodes; ++q) {
                if (q < rp.n) {
                    rows[0] = std::min(rows[0], rp.z[q]);
                    rows[1] = std::max(rows[1], rp.z[q] + 1);
                    // below L.total, which grid_info keeps under 2^31: fits an int
                    J.rnode.push_back((int)((int64_t)rp.z[q] * S.g.L.plane + (int64_t)rp.y[q] * S.g.L.pitch + rp.x[q]));
                    J.rw.push_back((float)rp.w[q]);
                } else {
                    J.rnode.push_back(0);
                    J.rw.push_back(0.f);
                }
            }
        }
        base += S.nrec;
        J.srows.push_back(rows[1] > rows[0] ? rows : std::array<int, 2>{0, 0});
        for (int r0 = 0; r0 < S.nrec; r0 += 64) J.stasks.push_back(SampleTask{s, r0});
        int slot = -1;
        for (int d = 0; d < (int)J.slot_shot.size(); ++d) {
            const ShotIn &o = J.shots[J.slot_shot[d]];
            if (o.v_pad == S.v_pad && o.g.NX == S.g.NX && o.g.NY == S.g.NY && o.g.NZ == S.g.NZ && o.g.h == S.g.h) {
                slot = d;
                break;
            }
        }
        if (slot < 0) {
            slot = (int)J.slot_shot.size();
            J.slot_shot.push_back(s);
        }
        J.dslot.push_back(slot);
    }
    const int ndim = J.shots[0].g.ndim;
    const bool persist = (J.flags & RTM_F_PERSISTENT) != 0;
    J.fw.ndim = J.rv.ndim = J.fw2.ndim = J.rv2.ndim = ndim;
    J.fw.tune = fit_tune(J, get_tune(0, ndim));
    if (persist) {
        // one strip per workgroup, one step per item
        J.fw.tune.tx = 1;
        J.fw.tune.steps = 1;
    }
    int rc = build_tiling(J, J.fw, false);
    if (rc) return rc;
    if (J.op != RTM_OP_MODEL) {
        // the storage reverse pass steps one field, as the forward pass does
        J.rv.tune = fit_tune(J, get_tune(J.op == RTM_OP_STORAGE ? 0 : 1, ndim));
        if (persist) {
            J.rv.tune.tx = 1;
            J.rv.tune.steps = 1;
        }
        rc = build_tiling(J, J.rv, true);
        if (rc) return rc;
    }
    J.pitems_f.clear();
    J.pitems_r.clear();
    J.pnum.clear();
    if (persist) {
        const int nsh = (int)J.shots.size();
        J.pnum.assign(2 * (size_t)nsh, 0);
        for (int t = 0; t < (int)J.fw.tiles.size(); ++t) {
            J.pitems_f.push_back(PItem{t, J.fw.tiles[t].shot});
            J.pnum[J.fw.tiles[t].shot]++;
        }
        if (J.op == RTM_OP_MODEL)
            for (int k = 0; k < (int)J.stasks.size(); ++k) {
                J.pitems_f.push_back(PItem{-1 - k, J.stasks[k].shot});
                J.pnum[J.stasks[k].shot]++;
            }
        for (int t = 0; t < (int)J.rv.tiles.size(); ++t) {
            J.pitems_r.push_back(PItem{t, J.rv.tiles[t].shot});
            J.pnum[nsh + J.rv.tiles[t].shot]++;
        }
    }
    // Multi-step tilings (2-D): the forward one for every op, the reverse
    // one for imaging (up to three steps) and the gradient (two).
    // Three steps per launch store the middle level only on the receiver
    // rows, so storage RTM (which copies whole stored levels) takes two.
    J.fw2 = Tiling{};
    J.rv2 = Tiling{};
    J.fw2.ndim = J.rv2.ndim = ndim;
    if (ndim == 2 && J.fw.tune.steps >= 2) {
        J.fw2.tune = J.fw.tune;
        J.fw2.steps = J.op == RTM_OP_STORAGE ? 2 : J.fw.tune.steps;
        if ((rc = build_tiling(J, J.fw2, false))) return rc;
    }
    if (ndim == 2 && (J.op == RTM_OP_RTM || J.op == RTM_OP_VJP) && J.rv.tune.steps >= 2) {
        J.rv2.tune = J.rv.tune;
        J.rv2.steps = J.op == RTM_OP_VJP ? 2 : J.rv.tune.steps;  // the gradient pass: two steps at most
        if ((rc = build_tiling(J, J.rv2, true))) return rc;
    }
    return RTM_OK;
}

Counts exact_counts(const Job &J)
{
    Counts c;
    c.tiles_f = J.fw.count();
    c.ents_f = J.fw.ents.size();
    c.cont_f = J.fw.cont.size();
    c.tiles_r = J.rv.count();
    c.ents_r = J.rv.ents.size();
    c.cont_r = J.rv.cont.size();
    c.tiles_f2 = J.fw2.count();
    c.ents_f2 = J.fw2.ents.size();
    c.cont_f2 = J.fw2.cont.size();
    c.tiles_r2 = J.rv2.count();
    c.ents_r2 = J.rv2.ents.size();
    c.cont_r2 = J.rv2.cont.size();
    c.stasks = J.stasks.size();
    c.rnode = J.rnode.size() / kMaxNodes;
    c.pitems_f = J.pitems_f.size();
    c.pitems_r = J.pitems_r.size();
    return c;
}

// Upper bounds for one shot, independent of positions and launch shape.
Counts bound_counts(const GridInfo &g, int op, int nrec)
{
    Counts c;
    c.tiles_f = max_tiles(g);
    c.ents_f = c.cont_f = kMaxNodes;
    if (op != RTM_OP_MODEL) {
        c.tiles_r = max_tiles(g);
        c.ents_r = c.cont_r = kMaxNodes + (int64_t)kMaxNodes * nrec;
    }
    if (g.ndim == 2) {
        // multi-step strips own >= 48 columns; a node lies in at most 2
        // strips x 3 tiles in z for the first step, 2 x 2 for the second
        // (three steps) and its owner: 11 entries
        const int64_t t2 = ((g.NX + 47) / 48) * (g.L.NZr / kMinZseg);
        c.tiles_f2 = t2;
        c.ents_f2 = c.cont_f2 = 11 * kMaxNodes;
        if (op == RTM_OP_RTM || op == RTM_OP_VJP) {
            c.tiles_r2 = t2;
            c.ents_r2 = c.cont_r2 = 11 * (kMaxNodes + (int64_t)kMaxNodes * nrec);
        }
    }
    c.stasks = (nrec + 63) / 64;
    c.rnode = nrec;
    return c;
}

// Device addresses of the job's buffers inside `ws`.
struct Dev {
    char *base;
    template <class T>
    T *at(size_t off) const { return (T *)(base + off); }
};

// Two shot tables: out[0 .. nsh) addresses the field sets in order, out[nsh
// .. 2 nsh) with the sets exchanged (current levels after an odd number of
// multi-step launches).
void fill_shot_devs(const Job &J, const Dev &D, std::vector<ShotDev> &out)
{
    const size_t nsh = J.shots.size();
    out.resize(2 * nsh);
    for (size_t i = 0; i < nsh; ++i) {
        const ShotIn &S = J.shots[i];
        ShotDev &d = out[i];
        std::memset(&d, 0, sizeof d);
        for (int k = 0; k < 8; ++k) d.fld[k] = J.ws.fld[i][k] ? D.at<float>(J.ws.fld[i][k]) : nullptr;
        d.acc0 = J.op == RTM_OP_MODEL ? nullptr : D.at<float>(J.ws.acc0[i]);
        d.acc1 = has_den(J.op) ? D.at<float>(J.ws.acc1[i]) : nullptr;
        d.Dp = D.at<float>(J.ws.dp[J.dslot[i]]);
        d.wav = S.wavelet;
        float *trint = D.at<float>(J.ws.trint[i]);
        d.sig = J.op == RTM_OP_MODEL ? nullptr : trint;
        d.rec_out = J.op == RTM_OP_MODEL ? trint : nullptr;
        d.rnode = D.at<int>(J.ws.rnode) + J.rbase[i] * kMaxNodes;
        d.rw = D.at<float>(J.ws.rw) + J.rbase[i] * kMaxNodes;
        d.nrec = S.nrec;
        d.ix0 = S.g.nb;
        d.ix1 = S.g.nb + (int)S.g.nx;
        d.iy0 = S.g.ndim == 3 ? S.g.nb : 0;
        d.iy1 = S.g.ndim == 3 ? S.g.nb + (int)S.g.ny : 1;
        d.iz0 = S.g.nb;
        d.iz1 = S.g.nb + (int)S.g.nz;
        d.sz0 = J.srows[i][0];
        d.sz1 = J.srows[i][1];
        d.L = S.g.L;
        ShotDev &x = out[nsh + i];
        x = d;
        for (int k = 0; k < 8; ++k) x.fld[k] = d.fld[k ^ 4];
    }
}

template <class T>
int upload(const Dev &D, size_t off, const std::vector<T> &v, hipStream_t st)
{
    if (v.empty()) return RTM_OK;
    RTM_HIP(hipMemcpyAsync(D.at<char>(off), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return RTM_OK;
}

// Copies the tables and shot descriptors into the workspace and, unless
// skipped, checks every D' slot's velocity range; synchronises once.
int job_upload_and_check(const Job &J, const Dev &D, std::vector<ShotDev> &shot_devs, hipStream_t st)
{
    int rc;
    fill_shot_devs(J, D, shot_devs);
    if ((rc = upload(D, J.ws.shots, shot_devs, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_f, J.fw.tiles, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_f, J.fw.tiles3, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_r, J.rv.tiles3, st))) return rc;
    if ((rc = upload(D, J.ws.ents_f, J.fw.ents, st))) return rc;
    if ((rc = upload(D, J.ws.cont_f, J.fw.cont, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_r, J.rv.tiles, st))) return rc;
    if ((rc = upload(D, J.ws.ents_r, J.rv.ents, st))) return rc;
    if ((rc = upload(D, J.ws.cont_r, J.rv.cont, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_f2, J.fw2.tiles, st))) return rc;
    if ((rc = upload(D, J.ws.ents_f2, J.fw2.ents, st))) return rc;
    if ((rc = upload(D, J.ws.cont_f2, J.fw2.cont, st))) return rc;
    if ((rc = upload(D, J.ws.tiles_r2, J.rv2.tiles, st))) return rc;
    if ((rc = upload(D, J.ws.ents_r2, J.rv2.ents, st))) return rc;
    if ((rc = upload(D, J.ws.cont_r2, J.rv2.cont, st))) return rc;
    if ((rc = upload(D, J.ws.stasks, J.stasks, st))) return rc;
    if ((rc = upload(D, J.ws.rnode, J.rnode, st))) return rc;
    if ((rc = upload(D, J.ws.rw, J.rw, st))) return rc;
    if (!J.pitems_f.empty()) {
        if ((rc = upload(D, J.ws.pitems_f, J.pitems_f, st))) return rc;
        if ((rc = upload(D, J.ws.pitems_r, J.pitems_r, st))) return rc;
        if ((rc = upload(D, J.ws.pnum, J.pnum, st))) return rc;
    }
    const int nslot = (int)J.slot_shot.size();
    std::vector<unsigned> vr(2 * (size_t)nslot, 0u);
    const bool check = !(J.flags & RTM_F_SKIP_CHECK);
    unsigned *scal = D.at<unsigned>(J.ws.scal);
    if (check) {
        for (int d = 0; d < nslot; ++d) {
            const GridInfo &g = J.shots[J.slot_shot[d]].g;
            RTM_HIP(launch_vrange(J.shots[J.slot_shot[d]].v_pad, (int64_t)g.NX * g.NY * g.NZ, scal + 64 + 2 * d, st));
        }
        RTM_HIP(hipMemcpyAsync(vr.data(), scal + 64, vr.size() * sizeof(unsigned), hipMemcpyDeviceToHost, st));
    }
    RTM_HIP(hipStreamSynchronize(st));
    if (check) {
        for (int d = 0; d < nslot; ++d) {
            const ShotIn &S = J.shots[J.slot_shot[d]];
            float vmax, vmin;
            std::memcpy(&vmax, &vr[2 * d], 4);
            std::memcpy(&vmin, &vr[2 * d + 1], 4);
            if (vr[2 * d] >= 0x7f800000u || !(vmin >= 0.f) || !(vmax > 0.f))
                return fail(RTM_ENUMERIC, "shot %d: velocity must be finite, >= 0 and not all 0 (max bits 0x%08x, min %g)",
                            J.slot_shot[d], vr[2 * d], (double)vmin);
            const double limit = std::sqrt(315.0 / (512.0 * S.g.ndim));
            const double courant = (double)vmax * J.dt / S.g.h;
            if (!(courant < limit))
                return fail(RTM_ECFL, "shot %d: max(v) dt / h = %.6f >= stability limit %.6f", J.slot_shot[d],
                            courant, limit);
        }
    }
    return RTM_OK;
}

// The device work of a job, after the upload (capturable in a hipGraph:
// kernel launches only).
int job_launch(const Job &J, const Dev &D, hipStream_t st, const rtm_probe_t *probe, bool timed)
{
    const ShotDev *table = D.at<ShotDev>(J.ws.shots);
    const int nsh = (int)J.shots.size();
    const int nt = J.nt;
    // Current shot table: 0 while the latest levels are in the first field
    // set, 1 after an odd number of multi-step launches.
    int cur = 0;
    auto SH = [&]() { return table + (size_t)cur * nsh; };
    auto fld_of = [&](int i, int k) { return D.at<float>(J.ws.fld[i][cur ? (k ^ 4) : k]); };
    unsigned *scal = D.at<unsigned>(J.ws.scal);
    // Two-step launches write the second field set: every level they touch
    // must have a buffer.
    for (int i = 0; i < nsh; ++i) {
        const bool need_p = J.fw2.steps > 1 || J.rv2.steps > 1, need_mu = J.rv2.steps > 1;
        const bool need_mid = J.op == RTM_OP_MODEL && J.fw2.steps == 3;
        if ((need_p && !(J.ws.fld[i][4] && J.ws.fld[i][5])) || (need_mu && !(J.ws.fld[i][6] && J.ws.fld[i][7])) ||
            (need_mid && !(J.ws.fld[i][2] && J.ws.fld[i][6])))
            return fail(RTM_EINVAL, "internal: shot %d lacks the second field set of multi-step launches", i);
    }
    for (int d = 0; d < (int)J.slot_shot.size(); ++d) {
        const ShotIn &S = J.shots[J.slot_shot[d]];
        RTM_HIP(launch_build_dp(S.g.L, S.v_pad, (float)(J.dt / S.g.h), D.at<float>(J.ws.dp[d]), st));
    }
    for (int i = 0; i < nsh; ++i) {
        const int64_t F = J.shots[i].g.L.total;
        for (int k = 0; k < 8; ++k)
            if (J.ws.fld[i][k]) RTM_HIP(launch_fill(D.at<float>(J.ws.fld[i][k]), F, 0.f, st));
        if (J.op != RTM_OP_MODEL) RTM_HIP(launch_fill(D.at<float>(J.ws.acc0[i]), F, 0.f, st));
        if (has_den(J.op)) RTM_HIP(launch_fill(D.at<float>(J.ws.acc1[i]), F, 0.f, st));
        if (J.op == RTM_OP_VJP && J.shots[i].grad_wavelet)
            RTM_HIP(launch_fill(D.at<float>(J.ws.wadj[i]), (int64_t)nt * kMaxNodes, 0.f, st));
        if (J.op != RTM_OP_MODEL)
            RTM_HIP(launch_transpose(J.shots[i].traces_in, D.at<float>(J.ws.trint[i]), J.shots[i].nrec, nt + 1, st));
    }
    // Forward pass (Algorithm 1; in RTM only the last two panels are kept).
    {
        const PassRange pass("rtm:forward");
        const bool sample = J.op == RTM_OP_MODEL;
        const Tile2D *tiles = D.at<Tile2D>(J.ws.tiles_f);
        const InjEnt *ents = D.at<InjEnt>(J.ws.ents_f);
        const Contrib *cont = D.at<Contrib>(J.ws.cont_f);
        const SampleTask *stasks = D.at<SampleTask>(J.ws.stasks);
        const int ntiles = J.fw.count();
        const int nsample = sample ? (int)J.stasks.size() : 0;
        const bool two = J.fw.ndim == 2 && J.fw2.steps > 1;
        const int fs = two ? J.fw2.steps : 1;
        const bool persist = !J.pitems_f.empty();
        LoopTimer timer(sample ? kLoopModelFwd : kLoopRtmFwd, persist ? 1 : nt / fs + nt % fs, st, timed);
        // Storage RTM: copy the interior of each stored level p^m once it
        // is current (before the step that overwrites p^{m-1} with p^{m+1}).
        auto keep = [&](int m) -> int {
            if (J.op != RTM_OP_STORAGE || m >= nt) return RTM_OK;
            const ShotIn &S = J.shots[0];
            if (m < S.phase || (m - S.phase) % S.stride != 0) return RTM_OK;
            const int64_t ncell = S.g.nx * S.g.ny * S.g.nz;
            RTM_HIP(launch_snap_store(SH(), 0, m & 1, ncell, S.snaps + (int64_t)((m - S.phase) / S.stride) * ncell,
                                      st));
            return RTM_OK;
        };
        int rc = RTM_OK;
        int n = 0;
        if (persist) {
            // every forward step in one launch; counters and status start at zero
            unsigned *cnt = D.at<unsigned>(J.ws.pcnt);
            RTM_HIP(launch_fill((float *)cnt, nsh + 1, 0.f, st));
            RTM_HIP(launch_fwd2d_persist(J.fw.tune.vec, SH(), tiles, D.at<PItem>(J.ws.pitems_f),
                                         (int)J.pitems_f.size(), D.at<int>(J.ws.pnum), ents, cont,
                                         sample ? stasks : nullptr, 0, nt, cnt, cnt + nsh, g_persist_wait_ms.load(),
                                         st));
            n = nt;
        }
        if (fs == 3) {
            // steps n .. n + 2 per launch; each launch records d^{n-2},
            // d^{n-1}, d^n (no stored levels: not for storage RTM)
            for (; n + 3 <= nt; n += 3) {
                RTM_HIP(launch_fwd2d_t3(J.fw2.tune.vec, SH(), D.at<Tile2D>(J.ws.tiles_f2), J.fw2.count(),
                                        J.fw2.nslots, D.at<InjEnt>(J.ws.ents_f2), D.at<Contrib>(J.ws.cont_f2),
                                        sample ? stasks : nullptr, nsample, n, st));
                cur ^= 1;
            }
            // the last launch's middle level (field 6 of the current table)
            // and level n - 1, which a one-step launch would overwrite
            if (sample && n >= 3) {
                RTM_HIP(launch_sample(SH(), stasks, nsample, n - 2, 6, st));
                RTM_HIP(launch_sample(SH(), stasks, nsample, n - 1, (n - 1) & 1, st));
            }
        } else if (two) {
            // steps n, n + 1 per launch; each launch records d^{n-1}, d^n
            for (; n + 2 <= nt; n += 2) {
                if ((rc = keep(n))) return rc;
                RTM_HIP(launch_fwd2d_t2(J.fw2.tune.vec, SH(), D.at<Tile2D>(J.ws.tiles_f2), J.fw2.count(),
                                        J.fw2.nslots, D.at<InjEnt>(J.ws.ents_f2), D.at<Contrib>(J.ws.cont_f2),
                                        sample ? stasks : nullptr, nsample, n, st));
                cur ^= 1;
                if ((rc = keep(n + 1))) return rc;
            }
            // an odd last step overwrites level n - 1: record it first
            if (sample && n < nt && n >= 1) RTM_HIP(launch_sample(SH(), stasks, nsample, n - 1, (n - 1) & 1, st));
        }
        for (; n < nt; ++n) {
            if ((rc = keep(n))) return rc;
            if (J.fw.ndim == 3)
                RTM_HIP(launch_fwd3d(J.fw.tune.vec, J.fw.tune.ty, SH(), (const Tile3D *)tiles, ntiles, J.fw.nslots,
                                     ents, cont, sample ? stasks : nullptr, nsample, n, st));
            else
                RTM_HIP(launch_fwd2d(J.fw.tune.vec, J.fw.tune.tx, SH(), tiles, ntiles, J.fw.nslots, ents, cont,
                                     sample ? stasks : nullptr, nsample, n, st));
        }
        timer.finish();
        if (sample) {
            if (fs == 2 && nt % 2 == 0 && nt >= 2)
                RTM_HIP(launch_sample(SH(), stasks, nsample, nt - 1, (nt - 1) & 1, st));
            RTM_HIP(launch_sample(SH(), stasks, nsample, nt, nt & 1, st));
        }
    }
    if (J.op == RTM_OP_MODEL) {
        for (int i = 0; i < nsh; ++i) {
            const ShotIn &S = J.shots[i];
            RTM_HIP(launch_transpose(D.at<float>(J.ws.trint[i]), S.traces_out, nt + 1, S.nrec, st));
            if (S.p_last) RTM_HIP(launch_unpack(S.g.L, fld_of(i, nt & 1), S.p_last, st));
            if (S.p_prev) RTM_HIP(launch_unpack(S.g.L, fld_of(i, (nt + 1) & 1), S.p_prev, st));
        }
        return RTM_OK;
    }
    // Reverse pass (Algorithm 3): mu^{nt} = D' h^2 R^T g^{nt}, mu^{nt+1} = 0,
    // then one fused launch per step k = nt-1 .. 0 (or per pair of steps).
    const PassRange pass(J.op == RTM_OP_VJP ? "rtm:reverse_grad" : "rtm:reverse_image");
    const bool grad = J.op == RTM_OP_VJP;
    const Tile2D *tiles = D.at<Tile2D>(J.ws.tiles_r);
    const InjEnt *ents = D.at<InjEnt>(J.ws.ents_r);
    const Contrib *cont = D.at<Contrib>(J.ws.cont_r);
    RTM_HIP(launch_inj_set(SH(), ents, J.rv.nsrc_ent, J.rv.nsrc_ent + J.rv.nrec_ent, cont, nt, st));
    const int ntiles = J.rv.count();
    if (J.op == RTM_OP_STORAGE) {
        // Algorithm 2: the receiver wavefield alone, imaging at the stored levels.
        const ShotIn &S = J.shots[0];
        const int64_t ncell = S.g.nx * S.g.ny * S.g.nz;
        LoopTimer timer(kLoopRevImage, nt, st, timed);
        for (int k = nt - 1; k >= 0; --k) {
            const bool stored = k >= S.phase && (k - S.phase) % S.stride == 0;
            const float *snap = stored ? S.snaps + (int64_t)((k - S.phase) / S.stride) * ncell : nullptr;
            if (J.rv.ndim == 3)
                RTM_HIP(launch_recv3d(J.rv.tune.vec, J.rv.tune.ty, SH(), (const Tile3D *)tiles, ntiles, J.rv.nslots,
                                      ents, cont, k, snap, st));
            else
                RTM_HIP(launch_recv2d(J.rv.tune.vec, J.rv.tune.tx, SH(), tiles, ntiles, J.rv.nslots, ents, cont, k,
                                      snap, st));
        }
        timer.finish();
        RTM_HIP(launch_image(SH(), 0, ncell, scal + 64 + 2 * J.slot_shot.size(), J.eps, S.image, 0, S.num, S.den,
                             st));
        return RTM_OK;
    }
    const int reinject = (J.flags & RTM_F_NO_REINJECT) ? 0 : 1;
    const bool probing = probe && probe->snap_k >= 0;
    const bool two = J.rv.ndim == 2 && J.rv2.steps > 1 && !probing;
    const int rs = two ? J.rv2.steps : 1;
    // wadj is recorded for a single-shot job only (its kernel argument is one
    // buffer); batched VJPs do not return wavelet gradients.
    float *wadj = (grad && nsh == 1 && J.shots[0].grad_wavelet) ? D.at<float>(J.ws.wadj[0]) : nullptr;
    const bool persist = !J.pitems_f.empty() && !probing;
    LoopTimer timer(grad ? kLoopRevGrad : kLoopRevImage, persist ? 1 : nt / rs + nt % rs, st, timed && !probing);
    int k = nt - 1;
    if (persist) {
        // every reverse step in one launch; the status word keeps the forward pass's
        unsigned *cnt = D.at<unsigned>(J.ws.pcnt);
        RTM_HIP(launch_fill((float *)cnt, nsh, 0.f, st));
        RTM_HIP(launch_rev2d_persist(J.rv.tune.vec, grad, SH(), tiles, D.at<PItem>(J.ws.pitems_r),
                                     (int)J.pitems_r.size(), D.at<int>(J.ws.pnum) + nsh, ents, cont, nt - 1, nt,
                                     reinject, wadj, cnt, cnt + nsh, g_persist_wait_ms.load(), st));
        k = -1;
    }
    if (rs == 3) {
        for (; k >= 2; k -= 3) {
            RTM_HIP(launch_rev2d_t3(J.rv2.tune.vec, SH(), D.at<Tile2D>(J.ws.tiles_r2), J.rv2.count(), J.rv2.nslots,
                                    D.at<InjEnt>(J.ws.ents_r2), D.at<Contrib>(J.ws.cont_r2), k, reinject, st));
            cur ^= 1;
        }
    } else if (two) {
        for (; k >= 1; k -= 2) {
            RTM_HIP(launch_rev2d_t2(J.rv2.tune.vec, grad, SH(), D.at<Tile2D>(J.ws.tiles_r2), J.rv2.count(),
                                    J.rv2.nslots, D.at<InjEnt>(J.ws.ents_r2), D.at<Contrib>(J.ws.cont_r2), k, reinject,
                                    wadj, st));
            cur ^= 1;
        }
    }
    for (; k >= 0; --k) {
        if (J.rv.ndim == 3)
            RTM_HIP(launch_rev3d(J.rv.tune.vec, J.rv.tune.ty, grad, SH(), (const Tile3D *)tiles, ntiles, J.rv.nslots,
                                 ents, cont, k, reinject, wadj, st));
        else
            RTM_HIP(launch_rev2d(J.rv.tune.vec, J.rv.tune.tx, grad, SH(), tiles, ntiles, J.rv.nslots, ents, cont, k,
                                 reinject, wadj, st));
        if (probing) {
            const ShotIn &S = J.shots[0];
            if (k - 1 == probe->snap_k && probe->snap_p)
                RTM_HIP(launch_unpack(S.g.L, fld_of(0, (k - 1) & 1), probe->snap_p, st));
            if (k == probe->snap_k && probe->snap_mu)
                RTM_HIP(launch_unpack(S.g.L, fld_of(0, 2 + (k & 1)), probe->snap_mu, st));
        }
    }
    timer.finish();
    // Finalisation, shot by shot (stream-ordered, so shots may share an
    // accumulated image buffer).
    for (int i = 0; i < nsh; ++i) {
        const ShotIn &S = J.shots[i];
        if (grad) {
            RTM_HIP(launch_grad(SH(), i, (int64_t)S.g.NX * S.g.NY * S.g.NZ, S.v_pad, (float)J.dt, S.grad_v_pad, st));
            if (S.grad_wavelet && nsh == 1)
                RTM_HIP(launch_wadj(D.at<float>(J.ws.wadj[i]), nt, (float)(1.0 / (S.g.h * S.g.h)), S.grad_wavelet, st));
        } else {
            RTM_HIP(launch_image(SH(), i, S.g.nx * S.g.ny * S.g.nz, scal + 64 + 2 * J.slot_shot.size() + i, J.eps,
                                 S.image, (J.flags & RTM_F_ACCUMULATE) ? 1 : 0, S.num, S.den, st));
        }
    }
    return RTM_OK;
}

int check_ws(const Job &J, void *ws, size_t ws_bytes)
{
    if (!ws) return fail(RTM_EWORKSPACE, "workspace is NULL (%zu bytes needed)", J.ws.bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(RTM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < J.ws.bytes) return fail(RTM_EWORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, J.ws.bytes);
    return RTM_OK;
}

// Eager execution of a job (single-shot entry points and plans without a graph).
int job_run(Job &J, void *ws, size_t ws_bytes, hipStream_t st, const rtm_probe_t *probe)
{
    int rc = check_ws(J, ws, ws_bytes);
    if (rc) return rc;
    Dev D{(char *)ws};
    std::vector<ShotDev> shot_devs;
    if ((rc = job_upload_and_check(J, D, shot_devs, st))) return rc;
    if ((rc = job_launch(J, D, st, probe, true))) return rc;
    if (!(J.flags & RTM_F_CHECK_FINITE)) return RTM_OK;
    // Outputs checked for NaN / Inf: an unstable run (or a non-finite input
    // that the velocity check does not cover, such as the wavelet or the
    // traces) is reported instead of returned silently.
    unsigned *flag = D.at<unsigned>(J.ws.scal);
    RTM_HIP(launch_fill((float *)flag, 1, 0.f, st));  // zero bits
    for (const ShotIn &S : J.shots) {
        const int64_t ni = S.g.nx * S.g.ny * S.g.nz, np = (int64_t)S.g.NX * S.g.NY * S.g.NZ;
        if (J.op == RTM_OP_MODEL) RTM_HIP(launch_nonfinite(S.traces_out, (int64_t)S.nrec * (J.nt + 1), flag, st));
        if (has_den(J.op)) RTM_HIP(launch_nonfinite(S.image, ni, flag, st));
        if (J.op == RTM_OP_VJP) RTM_HIP(launch_nonfinite(S.grad_v_pad, np, flag, st));
    }
    unsigned h = 0;
    RTM_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st));
    RTM_HIP(hipStreamSynchronize(st));
    if (h) return fail(RTM_ENUMERIC, "non-finite values in the output (unstable run or non-finite wavelet / traces)");
    return RTM_OK;
}

int check_common(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                 const float *src, int32_t nrec, const float *rec, GridInfo *g)
{
    int rc = grid_info(grid, g);
    if (rc) return rc;
    if (!v_pad) return fail(RTM_EINVAL, "v_pad is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RTM_EINVAL, "dt must be positive and finite");
    if (nt < 1) return fail(RTM_EINVAL, "nt must be >= 1");
    if (!wavelet) return fail(RTM_EINVAL, "wavelet is NULL");
    if (!src) return fail(RTM_EINVAL, "src is NULL");
    if (nrec < 1) return fail(RTM_EINVAL, "nrec must be >= 1");
    if (!rec) return fail(RTM_EINVAL, "rec is NULL");
    if ((int64_t)(nt + 1) * nrec >= ((int64_t)1 << 31)) return fail(RTM_EINVAL, "(nt + 1) * nrec too large");
    return RTM_OK;
}

// A one-shot job whose workspace layout uses position-independent bounds,
// so that rtm_workspace_bytes can size it without the acquisition.
int single_job(Job &J, int op, const GridInfo &g, const float *v_pad, double dt, int nt, const float *wavelet,
               const float *src, int nrec, const float *rec, uint32_t flags)
{
    J.op = op;
    J.nt = nt;
    J.dt = dt;
    J.flags = flags;
    ShotIn S;
    S.g = g;
    S.v_pad = v_pad;
    S.wavelet = wavelet;
    std::memcpy(S.src, src, sizeof S.src);
    S.nrec = nrec;
    S.rec.assign(rec, rec + 3 * (size_t)nrec);
    J.shots.push_back(std::move(S));
    int rc = build_job_tables(J);
    if (rc) return rc;
    J.ws = make_ws_layout(J, bound_counts(g, op, nrec));
    return RTM_OK;
}

size_t single_bytes(const GridInfo &g, int op, int nrec, int nt)
{
    Job J;
    J.op = op;
    J.nt = nt;
    ShotIn S;
    S.g = g;
    S.nrec = nrec;
    J.shots.push_back(S);
    J.slot_shot.push_back(0);
    J.dslot.push_back(0);
    return make_ws_layout(J, bound_counts(g, op, nrec)).bytes;
}

// Band options from the ABI struct: flags checked, taper table built on the
// host (Eqs. (4)-(5) in double, rounded once to FP32).
int band_opts(const GridInfo &g, const rtm_rbc_opts_t *o, BandOpts *b)
{
    std::memset(b, 0, sizeof *b);
    if (!o) return RTM_OK;
    if (o->flags & ~(RTM_RBC_TAPER | RTM_RBC_FREE_SURFACE)) return fail(RTM_EINVAL, "unknown band flags 0x%x", o->flags);
    b->flags = (o->flags & RTM_RBC_TAPER ? kBandTaper : 0u) | (o->flags & RTM_RBC_FREE_SURFACE ? kBandFreeSurface : 0u);
    if (o->flags & RTM_RBC_TAPER) {
        const double a = o->taper_alpha;
        if (!(a >= 0.0 && a <= 1.0)) return fail(RTM_EINVAL, "taper_alpha must be in [0, 1] (got %g)", a);
        if (g.nb > kMaxTaper) return fail(RTM_EINVAL, "taper needs nb <= %d (got %d)", kMaxTaper, g.nb);
        for (int i = 1; i <= g.nb; ++i) {
            if (g.nb == 1) {
                b->c[0] = 1.0f;
                break;
            }
            const double x = (double)i, n1 = (double)(g.nb - 1);
            const double lin = ((double)g.nb - x) / n1;                       // Eq. (4)
            const double gau = std::exp(-120.0 * (x - 1.0) * (x - 1.0) / (n1 * n1));  // Eq. (5)
            b->c[i - 1] = (float)(a * lin + (1.0 - a) * gau);
        }
    }
    return RTM_OK;
}

int pad_common(const rtm_grid_t *grid, const float *v_int, const rtm_rbc_opts_t *opts, const float *g_pad,
               float *out, void *ws, size_t ws_bytes, void *stream, bool adjoint)
{
    t_err.clear();
    GridInfo g;
    int rc = grid_info(grid, &g);
    if (rc) return rc;
    if (!v_int || !out || (adjoint && !g_pad)) return fail(RTM_EINVAL, "NULL array argument");
    if (!opts) return fail(RTM_EINVAL, "opts is NULL");
    BandOpts b;
    if ((rc = band_opts(g, opts, &b))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const unsigned *cap_bits = nullptr;
    if (!(opts->v_cap > 0.f)) {
        if (!ws || ws_bytes < 256 || ((uintptr_t)ws & 255))
            return fail(RTM_EWORKSPACE, "v_cap <= 0 needs an aligned workspace of 256 bytes");
        RTM_HIP(launch_vmax(v_int, g.nx * g.ny * g.nz, (unsigned *)ws, st));
        cap_bits = (const unsigned *)ws;
    }
    if (adjoint)
        RTM_HIP(launch_pad_adjoint(g.ndim, g.nb, g.nx, g.ny, g.nz, v_int, opts->seed, opts->v_cap, cap_bits, b, g_pad,
                                   out, st));
    else
        RTM_HIP(launch_rbc_pad(g.ndim, g.nb, g.nx, g.ny, g.nz, v_int, opts->seed, opts->v_cap, cap_bits, b, out, st));
    return RTM_OK;
}

}  // namespace

// ===========================================================================
// Batch plans
// ===========================================================================

struct rtm_plan {
    Job job;
};

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int rtm_abi_version(void) { return RTM_ABI_VERSION; }

const char *rtm_last_error(void) { return t_err.c_str(); }

int rtm_set_tuning(int op, int vec, int zseg)
{
    if (op == RTM_TUNE_EXACT || op == 0) {
        g_tune_exact = (op == RTM_TUNE_EXACT) ? (vec != 0) : 0;
        return RTM_OK;
    }
    if (vec != 1 && vec != 2 && vec != 4) return fail(RTM_EINVAL, "vec must be 1, 2 or 4");
    if (zseg < kMinZseg || zseg > 4095 || zseg % kZUnroll != 0)
        return fail(RTM_EINVAL, "zseg must be a multiple of %d in [%d, 4095]", kZUnroll, kMinZseg);
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    std::atomic<int> &g = op == RTM_OP_MODEL ? g_tune2d_fwd : g_tune2d_rev;
    g = (g.load() & ~0xffffff) | (vec << 16) | zseg;  // keeps the strips per workgroup
    return RTM_OK;
}

int rtm_set_tuning2d(int op, int vec, int tx, int zseg)
{
    if (vec != 1 && vec != 2 && vec != 4) return fail(RTM_EINVAL, "vec must be 1, 2 or 4");
    if (tx != 1 && tx != 2 && tx != 4) return fail(RTM_EINVAL, "tx must be 1, 2 or 4");
    if (zseg < kMinZseg || zseg > 4095 || zseg % kZUnroll != 0)
        return fail(RTM_EINVAL, "zseg must be a multiple of %d in [%d, 4095]", kZUnroll, kMinZseg);
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    std::atomic<int> &g = op == RTM_OP_MODEL ? g_tune2d_fwd : g_tune2d_rev;
    g = (g.load() & (0x3 << 28)) | (tx << 24) | (vec << 16) | zseg;  // keeps the steps per launch
    return RTM_OK;
}

int rtm_set_steps_per_launch(int op, int steps)
{
    if (steps < 1 || steps > 3) return fail(RTM_EINVAL, "steps must be 1, 2 or 3");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    std::atomic<int> &g = op == RTM_OP_MODEL ? g_tune2d_fwd : g_tune2d_rev;
    g = (g.load() & ~(0x3 << 28)) | ((steps - 1) << 28);
    return RTM_OK;
}

int rtm_get_steps_per_launch(int op, int *steps)
{
    if (!steps) return fail(RTM_EINVAL, "NULL output");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    *steps = get_tune(op == RTM_OP_MODEL ? 0 : 1, 2).steps;
    return RTM_OK;
}

int rtm_get_tuning2d(int op, int *vec, int *tx, int *zseg)
{
    if (!vec || !tx || !zseg) return fail(RTM_EINVAL, "NULL output");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    Tune t = get_tune(op == RTM_OP_MODEL ? 0 : 1, 2);
    *vec = t.vec;
    *tx = t.tx;
    *zseg = t.zseg;
    return RTM_OK;
}

int rtm_set_tuning3d(int op, int vec, int ty, int zseg)
{
    if (vec != 1 && vec != 2 && vec != 4) return fail(RTM_EINVAL, "vec must be 1, 2 or 4");
    if (ty != 4 && ty != 8 && ty != 16) return fail(RTM_EINVAL, "ty must be 4, 8 or 16");
    // 16-row workgroups (1024 threads, at most 128 registers a lane): the
    // forward update at vec 1 or 2, the fused reverse at vec 1 only.
    if (ty == 16 && (vec > 2 || (op != RTM_OP_MODEL && vec != 1)))
        return fail(RTM_EINVAL, "ty 16 needs vec 1 (reverse) or vec <= 2 (forward)");
    if (zseg < kMinZseg || zseg > 4095 || zseg % kZUnroll != 0)
        return fail(RTM_EINVAL, "zseg must be a multiple of %d in [%d, 4095]", kZUnroll, kMinZseg);
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    std::atomic<int> &g = op == RTM_OP_MODEL ? g_tune3d_fwd : g_tune3d_rev;
    g = (vec << 24) | (ty << 16) | (g.load() & (1 << 15)) | zseg;  // the tile order is kept
    return RTM_OK;
}

int rtm_set_tile_order3d(int op, int z_inner)
{
    if (z_inner != 0 && z_inner != 1) return fail(RTM_EINVAL, "z_inner must be 0 or 1");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    std::atomic<int> &g = op == RTM_OP_MODEL ? g_tune3d_fwd : g_tune3d_rev;
    g = (g.load() & ~(1 << 15)) | (z_inner << 15);
    return RTM_OK;
}

int rtm_get_tile_order3d(int op, int *z_inner)
{
    if (!z_inner) return fail(RTM_EINVAL, "NULL output");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    *z_inner = get_tune(op == RTM_OP_MODEL ? 0 : 1, 3).zin;
    return RTM_OK;
}

int rtm_get_tuning3d(int op, int *vec, int *ty, int *zseg)
{
    if (!vec || !ty || !zseg) return fail(RTM_EINVAL, "NULL output");
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    Tune t = get_tune(op == RTM_OP_MODEL ? 0 : 1, 3);
    *vec = t.vec;
    *ty = t.ty;
    *zseg = t.zseg;
    return RTM_OK;
}

int rtm_get_tuning(int op, int *vec, int *zseg)
{
    if (!vec || !zseg) return fail(RTM_EINVAL, "NULL output");
    if (op == RTM_TUNE_EXACT) {
        *vec = g_tune_exact.load();
        *zseg = 0;
        return RTM_OK;
    }
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    Tune t = get_tune(op == RTM_OP_MODEL ? 0 : 1, 2);
    *vec = t.vec;
    *zseg = t.zseg;
    return RTM_OK;
}

int rtm_set_persist_wait(double ms)
{
    if (!(ms >= 0.0) || !(ms <= 3.6e6)) return fail(RTM_EINVAL, "wait limit must be in [0, 3.6e6] ms");
    g_persist_wait_ms = ms;
    return RTM_OK;
}

int rtm_get_persist_wait(double *ms)
{
    if (!ms) return fail(RTM_EINVAL, "NULL output");
    *ms = g_persist_wait_ms.load();
    return RTM_OK;
}

int rtm_timing_enable(int on)
{
    g_timing_on = on ? 1 : 0;
    return RTM_OK;
}

int rtm_timing_read(double *ms, int64_t *launches)
{
    if (!ms || !launches) return fail(RTM_EINVAL, "NULL output");
    for (int k = 0; k < kLoopKinds; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    std::vector<PendingTiming> pend;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        pend.swap(g_timing_pending);
    }
    int rc = RTM_OK;
    for (auto &p : pend) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, p.start, p.stop);
        if (e == hipSuccess) {
            ms[p.kind] += t;
            launches[p.kind] += p.launches;
        } else {
            rc = fail(RTM_EHIP, "event timing: %s", hipGetErrorString(e));
        }
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    return rc;
}

int rtm_workspace_bytes(const rtm_grid_t *grid, int op, int32_t nrec, int32_t nt, size_t *bytes)
{
    t_err.clear();
    GridInfo g;
    int rc = grid_info(grid, &g);
    if (rc) return rc;
    if (!bytes) return fail(RTM_EINVAL, "bytes is NULL");
    if (op < RTM_OP_RBC_PAD || op > RTM_OP_STORAGE) return fail(RTM_EINVAL, "unknown op %d", op);
    if (op == RTM_OP_RBC_PAD) {
        *bytes = 256;
        return RTM_OK;
    }
    if (nrec < 1 || nt < 1) return fail(RTM_EINVAL, "nrec and nt must be >= 1");
    *bytes = single_bytes(g, op, nrec, nt);
    return RTM_OK;
}

int rtm_rbc_pad_ex(const rtm_grid_t *grid, const float *v_int, const rtm_rbc_opts_t *opts, float *v_pad, void *ws,
                   size_t ws_bytes, void *stream)
{
    return pad_common(grid, v_int, opts, nullptr, v_pad, ws, ws_bytes, stream, false);
}

int rtm_pad_adjoint_ex(const rtm_grid_t *grid, const float *v_int, const rtm_rbc_opts_t *opts, const float *grad_v_pad,
                       float *grad_v_int, void *ws, size_t ws_bytes, void *stream)
{
    return pad_common(grid, v_int, opts, grad_v_pad, grad_v_int, ws, ws_bytes, stream, true);
}

int rtm_rbc_pad(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap, float *v_pad, void *ws,
                size_t ws_bytes, void *stream)
{
    const rtm_rbc_opts_t o{seed, v_cap, 0u, 0.0};
    return pad_common(grid, v_int, &o, nullptr, v_pad, ws, ws_bytes, stream, false);
}

int rtm_pad_adjoint(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap, const float *grad_v_pad,
                    float *grad_v_int, void *ws, size_t ws_bytes, void *stream)
{
    const rtm_rbc_opts_t o{seed, v_cap, 0u, 0.0};
    return pad_common(grid, v_int, &o, grad_v_pad, grad_v_int, ws, ws_bytes, stream, true);
}

int rtm_model_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                   const float *src, int32_t nrec, const float *rec, float *traces, float *p_last, float *p_prev,
                   uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = check_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, &g);
    if (rc) return rc;
    if (!traces) return fail(RTM_EINVAL, "traces is NULL");
    Job J;
    if ((rc = single_job(J, RTM_OP_MODEL, g, v_pad, dt, nt, wavelet, src, nrec, rec, flags))) return rc;
    J.shots[0].traces_out = traces;
    J.shots[0].p_last = p_last;
    J.shots[0].p_prev = p_prev;
    return job_run(J, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

int rtm_rtm_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                 const float *src, int32_t nrec, const float *rec, const float *traces, float eps_rel, float *image,
                 float *num, float *den, const rtm_probe_t *probe, uint32_t flags, void *ws, size_t ws_bytes,
                 void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = check_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, &g);
    if (rc) return rc;
    if (!traces) return fail(RTM_EINVAL, "traces is NULL");
    if (!image) return fail(RTM_EINVAL, "image is NULL");
    if (!(eps_rel >= 0.f) || !std::isfinite(eps_rel)) return fail(RTM_EINVAL, "eps_rel must be finite and >= 0");
    if (probe && probe->snap_k >= 0 && probe->snap_k > nt - 2)
        return fail(RTM_EINVAL, "probe step %d outside [0, nt - 2]", (int)probe->snap_k);
    Job J;
    if ((rc = single_job(J, RTM_OP_RTM, g, v_pad, dt, nt, wavelet, src, nrec, rec, flags & ~RTM_F_ACCUMULATE)))
        return rc;
    J.eps = eps_rel;
    J.shots[0].traces_in = traces;
    J.shots[0].image = image;
    J.shots[0].num = num;
    J.shots[0].den = den;
    return job_run(J, ws, ws_bytes, (hipStream_t)stream, probe);
}

int rtm_nyquist_stride(double dt, double f_max, double f_min, int32_t *stride)
{
    t_err.clear();
    if (!stride) return fail(RTM_EINVAL, "stride is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RTM_EINVAL, "dt must be positive and finite");
    if (!(f_min >= 0.0) || !(f_max > f_min) || !std::isfinite(f_max))
        return fail(RTM_EINVAL, "need 0 <= f_min < f_max, finite (got %g, %g)", f_min, f_max);
    // Eq. (7); the small allowance keeps exact ratios such as 5 ms / 0.5 ms at 10
    const double ratio = 1.0 / (2.0 * (f_max - f_min) * dt);
    const double steps = std::floor(ratio * (1.0 + 1e-12));
    *stride = (int32_t)std::max(1.0, std::min(steps, 1073741824.0));
    return RTM_OK;
}

int rtm_storage_count(int32_t nt, int32_t stride, int32_t phase, int64_t *count)
{
    t_err.clear();
    if (!count) return fail(RTM_EINVAL, "count is NULL");
    if (nt < 1) return fail(RTM_EINVAL, "nt must be >= 1");
    if (stride < 1 || phase < 0 || phase >= stride)
        return fail(RTM_EINVAL, "need stride >= 1 and 0 <= phase < stride (got %d, %d)", (int)stride, (int)phase);
    *count = phase < nt ? (int64_t)(nt - 1 - phase) / stride + 1 : 0;
    return RTM_OK;
}

int rtm_storage_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                     const float *src, int32_t nrec, const float *rec, const float *traces, int32_t stride,
                     int32_t phase, float eps_rel, float *image, float *num, float *den, float *snapshots,
                     size_t snapshot_bytes, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = check_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, &g);
    if (rc) return rc;
    if (!traces) return fail(RTM_EINVAL, "traces is NULL");
    if (!image) return fail(RTM_EINVAL, "image is NULL");
    if (!(eps_rel >= 0.f) || !std::isfinite(eps_rel)) return fail(RTM_EINVAL, "eps_rel must be finite and >= 0");
    int64_t count = 0;
    if ((rc = rtm_storage_count(nt, stride, phase, &count))) return rc;
    const int64_t ncell = g.nx * g.ny * g.nz;
    if (count > 0 && !snapshots) return fail(RTM_EINVAL, "snapshots is NULL");
    if ((double)count * (double)ncell * 4.0 > (double)snapshot_bytes)
        return fail(RTM_EINVAL, "snapshots: %lld levels of %lld cells need %.0f bytes, %zu given", (long long)count,
                    (long long)ncell, (double)count * (double)ncell * 4.0, snapshot_bytes);
    if (flags & ~(RTM_F_SKIP_CHECK | RTM_F_CHECK_FINITE))
        return fail(RTM_EINVAL, "unsupported flags 0x%x", (unsigned)flags);
    Job J;
    if ((rc = single_job(J, RTM_OP_STORAGE, g, v_pad, dt, nt, wavelet, src, nrec, rec, flags))) return rc;
    J.eps = eps_rel;
    ShotIn &S = J.shots[0];
    S.traces_in = traces;
    S.image = image;
    S.num = num;
    S.den = den;
    S.snaps = snapshots;
    S.stride = stride;
    S.phase = phase;
    return job_run(J, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

int rtm_model_shot_vjp(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                       const float *src, int32_t nrec, const float *rec, const float *grad_traces, float *grad_v_pad,
                       float *grad_wavelet, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = check_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, &g);
    if (rc) return rc;
    if (!grad_traces) return fail(RTM_EINVAL, "grad_traces is NULL");
    if (!grad_v_pad) return fail(RTM_EINVAL, "grad_v_pad is NULL");
    Job J;
    if ((rc = single_job(J, RTM_OP_VJP, g, v_pad, dt, nt, wavelet, src, nrec, rec, flags & ~RTM_F_NO_REINJECT)))
        return rc;
    J.shots[0].traces_in = grad_traces;
    J.shots[0].grad_v_pad = grad_v_pad;
    J.shots[0].grad_wavelet = grad_wavelet;
    return job_run(J, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

int rtm_batch_plan(int op, int32_t nshots, const rtm_shot_desc_t *descs, double dt, int32_t nt, float eps_rel,
                   uint32_t flags, rtm_plan_t **plan, size_t *ws_bytes)
{
    t_err.clear();
    if (!plan || !ws_bytes) return fail(RTM_EINVAL, "plan and ws_bytes must be non-NULL");
    *plan = nullptr;
    if (op != RTM_OP_MODEL && op != RTM_OP_RTM && op != RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    if (nshots < 1 || !descs) return fail(RTM_EINVAL, "need at least one shot");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RTM_EINVAL, "dt must be positive and finite");
    if (nt < 1) return fail(RTM_EINVAL, "nt must be >= 1");
    if (op == RTM_OP_RTM && (!(eps_rel >= 0.f) || !std::isfinite(eps_rel)))
        return fail(RTM_EINVAL, "eps_rel must be finite and >= 0");
    if ((flags & RTM_F_PERSISTENT) && (flags & RTM_F_GRAPH))
        return fail(RTM_EINVAL, "RTM_F_PERSISTENT checks its run's status and cannot be combined with RTM_F_GRAPH");
    if ((flags & RTM_F_PERSISTENT) && descs[0].grid.ndim != 2)
        return fail(RTM_EINVAL, "RTM_F_PERSISTENT is implemented for 2-D shots");
    rtm_plan *P = new (std::nothrow) rtm_plan;
    if (!P) return fail(RTM_EINVAL, "out of host memory");
    Job &J = P->job;
    J.op = op;
    J.nt = nt;
    J.dt = dt;
    J.eps = eps_rel;
    J.flags = flags;
    for (int s = 0; s < nshots; ++s) {
        const rtm_shot_desc_t &d = descs[s];
        ShotIn S;
        int rc = grid_info(&d.grid, &S.g);
        if (!rc && s > 0 && S.g.ndim != J.shots[0].g.ndim)
            rc = fail(RTM_EINVAL, "shot %d: all shots of a batch must have the same dimension", s);
        if (!rc && (!d.v_pad || !d.wavelet)) rc = fail(RTM_EINVAL, "shot %d: v_pad and wavelet are required", s);
        if (!rc && (d.nrec < 1 || !d.rec)) rc = fail(RTM_EINVAL, "shot %d: at least one receiver is required", s);
        if (!rc && (int64_t)(nt + 1) * d.nrec >= ((int64_t)1 << 31)) rc = fail(RTM_EINVAL, "shot %d: too many samples", s);
        if (!rc && op == RTM_OP_MODEL && !d.traces_out) rc = fail(RTM_EINVAL, "shot %d: traces_out is required", s);
        if (!rc && op != RTM_OP_MODEL && !d.traces_in) rc = fail(RTM_EINVAL, "shot %d: traces_in is required", s);
        if (!rc && op == RTM_OP_RTM && !d.image) rc = fail(RTM_EINVAL, "shot %d: image is required", s);
        if (!rc && op == RTM_OP_VJP && !d.grad_v_pad) rc = fail(RTM_EINVAL, "shot %d: grad_v_pad is required", s);
        if (rc) {
            delete P;
            return rc;
        }
        S.v_pad = d.v_pad;
        S.wavelet = d.wavelet;
        std::memcpy(S.src, d.src, sizeof S.src);
        S.nrec = d.nrec;
        S.rec.assign(d.rec, d.rec + 3 * (size_t)d.nrec);
        S.traces_in = d.traces_in;
        S.traces_out = d.traces_out;
        S.image = d.image;
        S.grad_v_pad = d.grad_v_pad;
        J.shots.push_back(std::move(S));
    }
    int rc = build_job_tables(J);
    if (rc) {
        delete P;
        return rc;
    }
    J.ws = make_ws_layout(J, exact_counts(J));
    *ws_bytes = J.ws.bytes;
    *plan = P;
    return RTM_OK;
}

int rtm_batch_run(rtm_plan_t *plan, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    if (!plan) return fail(RTM_EINVAL, "plan is NULL");
    Job &J = plan->job;
    hipStream_t st = (hipStream_t)stream;
    int rc = check_ws(J, ws, ws_bytes);
    if (rc) return rc;
    Dev D{(char *)ws};
    std::vector<ShotDev> shot_devs;
    if ((rc = job_upload_and_check(J, D, shot_devs, st))) return rc;
    if (J.flags & RTM_F_PERSISTENT) {
        if ((rc = job_launch(J, D, st, nullptr, true))) return rc;
        unsigned status = 0;
        RTM_HIP(hipMemcpyAsync(&status, D.at<unsigned>(J.ws.pcnt) + J.shots.size(), sizeof status,
                               hipMemcpyDeviceToHost, st));
        RTM_HIP(hipStreamSynchronize(st));
        if (status)
            return fail(RTM_EHIP, "persistent run stopped: a workgroup waited more than %g ms for its shot's "
                                  "previous step (not all workgroups resident?); outputs are invalid",
                        g_persist_wait_ms.load());
        return RTM_OK;
    }
    if (!(J.flags & RTM_F_GRAPH)) return job_launch(J, D, st, nullptr, true);
    if (!st) return fail(RTM_EINVAL, "RTM_F_GRAPH needs a non-NULL stream (the NULL stream cannot be captured)");
    if (J.gexec && (J.g_ws != ws || J.g_st != st)) {
        (void)hipGraphExecDestroy(J.gexec);
        J.gexec = nullptr;
    }
    if (!J.gexec) {
        hipGraph_t graph = nullptr;
        RTM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        rc = job_launch(J, D, st, nullptr, false);
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(RTM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&J.gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            J.gexec = nullptr;
            return fail(RTM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        J.g_ws = ws;
        J.g_st = st;
    }
    RTM_HIP(hipGraphLaunch(J.gexec, st));
    return RTM_OK;
}

int rtm_window_extract(int64_t nz, int64_t nx_global, int64_t x0, int64_t width, const float *global, float *window,
                       void *stream)
{
    t_err.clear();
    if (nz < 1 || nx_global < 1 || width < 1 || x0 < 0 || x0 + width > nx_global)
        return fail(RTM_EINVAL, "window [%lld, %lld) outside [0, %lld)", (long long)x0, (long long)(x0 + width),
                    (long long)nx_global);
    if (!global || !window) return fail(RTM_EINVAL, "NULL array");
    RTM_HIP(launch_window((float *)global, nullptr, window, nz, nx_global, x0, width, 0, (hipStream_t)stream));
    return RTM_OK;
}

int rtm_window_accumulate(int64_t nz, int64_t nx_global, int64_t x0, int64_t width, const float *window,
                          float *global, void *stream)
{
    t_err.clear();
    if (nz < 1 || nx_global < 1 || width < 1 || x0 < 0 || x0 + width > nx_global)
        return fail(RTM_EINVAL, "window [%lld, %lld) outside [0, %lld)", (long long)x0, (long long)(x0 + width),
                    (long long)nx_global);
    if (!global || !window) return fail(RTM_EINVAL, "NULL array");
    RTM_HIP(launch_window(global, window, nullptr, nz, nx_global, x0, width, 1, (hipStream_t)stream));
    return RTM_OK;
}

int rtm_misfit_ws_bytes(size_t *bytes)
{
    if (!bytes) return fail(RTM_EINVAL, "bytes is NULL");
    *bytes = align256(misfit_ws_bytes());
    return RTM_OK;
}

int rtm_l2_misfit(int64_t n, const float *d, const float *d_obs, float *residual, double *J, void *ws,
                  size_t ws_bytes, void *stream)
{
    t_err.clear();
    if (n < 1 || !d || !d_obs || !J) return fail(RTM_EINVAL, "bad arguments");
    if (!ws || ws_bytes < misfit_ws_bytes() || ((uintptr_t)ws & 255))
        return fail(RTM_EWORKSPACE, "misfit workspace of %zu aligned bytes needed", misfit_ws_bytes());
    RTM_HIP(launch_misfit(d, d_obs, residual, n, ws, J, (hipStream_t)stream));
    return RTM_OK;
}

int rtm_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu, void *stream)
{
    t_err.clear();
    if (!src || !dst) return fail(RTM_EINVAL, "NULL buffer");
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15) || (bytes & 15))
        return fail(RTM_EINVAL, "buffers and size must be multiples of 16 bytes");
    if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(RTM_EINVAL, "blocks_per_cu must be in [1, 64]");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (a < b + bytes && b < a + bytes && bytes > 0) return fail(RTM_EINVAL, "buffers overlap");
    RTM_HIP(launch_stream_copy(src, dst, (int64_t)(bytes / 16), blocks_per_cu, (hipStream_t)stream));
    return RTM_OK;
}

int rtm_batch_free(rtm_plan_t *plan)
{
    if (!plan) return RTM_OK;
    if (plan->job.gexec) (void)hipGraphExecDestroy(plan->job.gexec);
    delete plan;
    return RTM_OK;
}

}  // extern "C"
