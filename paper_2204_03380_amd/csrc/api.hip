// Host runtime of librtm: argument validation, acquisition tables,
// workspace carving and the launch sequences behind the C ABI of
// include/rtm.h.  Every device buffer comes from the caller.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "rtm.h"

namespace rtm {
// prop2d.hip
hipError_t launch_fwd2d(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st);
hipError_t launch_rev2d(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st);
// aux.hip
hipError_t launch_vrange(const float *v, int64_t n, unsigned *maxmin2, hipStream_t st);
hipError_t launch_vmax(const float *v, int64_t n, unsigned *out, hipStream_t st);
hipError_t launch_rbc_pad(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int, uint64_t seed,
                          float v_cap, const unsigned *cap_bits, float *v_pad, hipStream_t st);
hipError_t launch_pad_adjoint(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int,
                              uint64_t seed, float v_cap, const unsigned *cap_bits, const float *g_pad,
                              float *g_int, hipStream_t st);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_build_dp(const Layout &L, const float *v_pad, float dt_over_h, float *Dp, hipStream_t st);
hipError_t launch_unpack(const Layout &L, const float *f, float *out, hipStream_t st);
hipError_t launch_transpose(const float *in, float *out, int64_t R, int64_t C, hipStream_t st);
hipError_t launch_inj_set(const ShotDev *shots, int shot, const InjEnt *ents, int ebeg, int eend,
                          const Contrib *cont, int step, hipStream_t st);
hipError_t launch_sample(const ShotDev *shots, const SampleTask *stasks, int ntask, int n, hipStream_t st);
hipError_t launch_image(const ShotDev *shots, int shot, int64_t ninterior, unsigned *dmax_bits, float eps_rel,
                        float *image, float *num, float *den, hipStream_t st);
hipError_t launch_grad(const ShotDev *shots, int shot, int64_t npad, const float *v_pad, float dt, float *grad,
                       hipStream_t st);
hipError_t launch_wadj(const float *parts, int nt, float scale, float *out, hipStream_t st);
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
};

std::atomic<int> g_tune2d_fwd{(1 << 16) | 16};
std::atomic<int> g_tune2d_rev{(1 << 16) | 16};

Tune get_tune(int which)
{
    int v = (which == 0 ? g_tune2d_fwd : g_tune2d_rev).load();
    return Tune{v >> 16, v & 0xffff};
}

constexpr int kMinZseg = 4;

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
// Workspace carving
// ---------------------------------------------------------------------------

struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Device buffers of one single-shot call.
struct ShotBufs {
    float *Dp = nullptr;
    float *fld[4] = {nullptr, nullptr, nullptr, nullptr};
    float *acc0 = nullptr, *acc1 = nullptr;
    float *traces = nullptr;  // [nt + 1][nrec]
    float *wadj = nullptr;    // [nt][kMaxNodes]
    ShotDev *shot = nullptr;
    Tile2D *tiles = nullptr;
    InjEnt *ents = nullptr;
    Contrib *cont = nullptr;
    SampleTask *stasks = nullptr;
    int *rnode = nullptr;
    float *rw = nullptr;
    unsigned *scal = nullptr;  // 4 words of scratch
    size_t bytes = 0;
};

int max_tiles(const GridInfo &g)
{
    return (int)(((int64_t)(g.NX + 63) / 64) * ((g.NZ + kMinZseg - 1) / kMinZseg));
}

ShotBufs carve(void *ws, const GridInfo &g, int op, int nrec, int nt)
{
    Carve c(ws);
    ShotBufs b;
    const int64_t F = g.L.total;
    b.scal = c.take<unsigned>(64);
    if (op != RTM_OP_RBC_PAD) {
        b.Dp = c.take<float>(F);
        int nf = (op == RTM_OP_MODEL) ? 2 : 4;
        for (int i = 0; i < nf; ++i) b.fld[i] = c.take<float>(F);
        if (op == RTM_OP_RTM) {
            b.acc0 = c.take<float>(F);
            b.acc1 = c.take<float>(F);
        } else if (op == RTM_OP_VJP) {
            b.acc0 = c.take<float>(F);
            b.wadj = c.take<float>((size_t)nt * kMaxNodes);
        }
        b.traces = c.take<float>((size_t)(nt + 1) * (size_t)nrec);
        b.shot = c.take<ShotDev>(1);
        int mt = max_tiles(g);
        b.tiles = c.take<Tile2D>(mt);
        int ment = kMaxNodes + kMaxNodes * nrec;
        b.ents = c.take<InjEnt>(ment);
        b.cont = c.take<Contrib>(ment);
        b.stasks = c.take<SampleTask>((nrec + 63) / 64 + 1);
        b.rnode = c.take<int>((size_t)nrec * kMaxNodes);
        b.rw = c.take<float>((size_t)nrec * kMaxNodes);
    }
    b.bytes = c.off;
    return b;
}

// ---------------------------------------------------------------------------
// Acquisition tables (host side) for one shot on the 2-D tiling
// ---------------------------------------------------------------------------

struct HostTables {
    std::vector<Tile2D> tiles;
    std::vector<InjEnt> ents;
    std::vector<Contrib> cont;
    std::vector<SampleTask> stasks;
    std::vector<int> rnode;
    std::vector<float> rw;
    int nsrc_ent = 0, nrec_ent = 0;  // ents = [source entries][receiver entries]
    int nslots = 0;
};

struct RawEnt {
    int tile, z, y, x;
    std::vector<Contrib> c;
    int slot;
};

int build_tables_2d(const GridInfo &g, Tune tune, const float *src, int nrec, const float *rec, HostTables *T)
{
    const int strip = 64 * tune.vec;
    const int ns = (g.NX + strip - 1) / strip;
    const int nzs = (g.NZ + tune.zseg - 1) / tune.zseg;
    T->tiles.clear();
    for (int s = 0; s < ns; ++s)
        for (int zs = 0; zs < nzs; ++zs) {
            Tile2D t{};
            t.shot = 0;
            t.x0 = s * strip;
            t.z0 = zs * tune.zseg;
            t.z1 = std::min(t.z0 + tune.zseg, g.NZ);
            T->tiles.push_back(t);
        }
    auto tile_of = [&](int z, int x) { return (x / strip) * nzs + z / tune.zseg; };

    PointOp sp;
    if (!make_point(g, src, &sp))
        return fail(RTM_ERANGE, "source (%g, %g, %g) outside the interior", src[0], src[1], src[2]);
    const double hd = std::pow(g.h, g.ndim);
    const double h2 = g.h * g.h;
    std::vector<RawEnt> se, re;
    for (int q = 0; q < sp.n; ++q) {
        RawEnt e{tile_of(sp.z[q], sp.x[q]), sp.z[q], sp.y[q], sp.x[q], {}, q};
        // s = W h^2 / h^d: the source term D (B w) expressed with D' = D / h^2.
        e.c.push_back(Contrib{0, (float)(sp.w[q] * h2 / hd)});
        se.push_back(e);
    }
    std::map<std::tuple<int, int, int>, size_t> node_of;
    T->rnode.assign((size_t)nrec * kMaxNodes, 0);
    T->rw.assign((size_t)nrec * kMaxNodes, 0.f);
    for (int r = 0; r < nrec; ++r) {
        PointOp rp;
        if (!make_point(g, rec + 3 * (size_t)r, &rp))
            return fail(RTM_ERANGE, "receiver %d (%g, %g, %g) outside the interior", r, rec[3 * r], rec[3 * r + 1],
                        rec[3 * r + 2]);
        for (int q = 0; q < rp.n; ++q) {
            T->rnode[(size_t)r * kMaxNodes + q] =
                (int)((int64_t)rp.z[q] * g.L.plane + (int64_t)rp.y[q] * g.L.pitch + rp.x[q]);
            T->rw[(size_t)r * kMaxNodes + q] = (float)rp.w[q];
            auto key = std::make_tuple(rp.z[q], rp.y[q], rp.x[q]);
            auto it = node_of.find(key);
            if (it == node_of.end()) {
                node_of[key] = re.size();
                re.push_back(RawEnt{tile_of(rp.z[q], rp.x[q]), rp.z[q], rp.y[q], rp.x[q], {}, 0});
                it = node_of.find(key);
            }
            // Receiver injection D R^T g = D' h^2 W g.
            re[it->second].c.push_back(Contrib{r, (float)(rp.w[q] * h2)});
        }
    }
    auto order = [](const RawEnt &a, const RawEnt &b) {
        return std::tie(a.tile, a.z, a.y, a.x) < std::tie(b.tile, b.z, b.y, b.x);
    };
    std::sort(se.begin(), se.end(), order);
    std::sort(re.begin(), re.end(), order);
    T->ents.clear();
    T->cont.clear();
    for (auto &t : T->tiles) t.sbeg = t.send = t.rbeg = t.rend = 0;
    auto emit = [&](std::vector<RawEnt> &v, bool is_src) {
        for (auto &e : v) {
            InjEnt E{e.z, e.y, e.x, (int)T->cont.size(), 0, e.slot};
            for (auto &c : e.c) T->cont.push_back(c);
            E.cend = (int)T->cont.size();
            int idx = (int)T->ents.size();
            T->ents.push_back(E);
            Tile2D &t = T->tiles[e.tile];
            if (is_src) {
                if (t.send == t.sbeg) t.sbeg = idx;
                t.send = idx + 1;
            } else {
                if (t.rend == t.rbeg) t.rbeg = idx;
                t.rend = idx + 1;
            }
        }
    };
    emit(se, true);
    T->nsrc_ent = (int)se.size();
    emit(re, false);
    T->nrec_ent = (int)re.size();
    T->stasks.clear();
    for (int r0 = 0; r0 < nrec; r0 += 64) T->stasks.push_back(SampleTask{0, r0});
    const int nt_ = (int)T->tiles.size();
    T->nslots = (nt_ + kNumXcd - 1) / kNumXcd * kNumXcd;
    return RTM_OK;
}

// ---------------------------------------------------------------------------
// Common call preparation
// ---------------------------------------------------------------------------

struct Prepared {
    GridInfo g;
    ShotBufs b;
    HostTables T;
    Tune tune;
    hipStream_t st;
};

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

// Validates the workspace, builds and uploads the tables, checks the
// velocity model (unless skipped) and synchronises the stream once.
int prepare(const GridInfo &g, int op, const float *v_pad, double dt, int32_t nt, const float *src, int32_t nrec,
            const float *rec, uint32_t flags, void *ws, size_t ws_bytes, void *stream, Prepared *P)
{
    P->g = g;
    P->st = (hipStream_t)stream;
    P->tune = get_tune(op == RTM_OP_MODEL ? 0 : 1);
    if (g.ndim != 2) return fail(RTM_EINVAL, "3-D propagation is not available in this build");
    ShotBufs need = carve(nullptr, g, op, nrec, nt);
    if (!ws) return fail(RTM_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need.bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(RTM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need.bytes) return fail(RTM_EWORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, need.bytes);
    int rc = build_tables_2d(g, P->tune, src, nrec, rec, &P->T);
    if (rc) return rc;
    P->b = carve(ws, g, op, nrec, nt);
    hipStream_t st = P->st;
    const HostTables &T = P->T;
    RTM_HIP(hipMemcpyAsync(P->b.tiles, T.tiles.data(), T.tiles.size() * sizeof(Tile2D), hipMemcpyHostToDevice, st));
    if (!T.ents.empty()) {
        RTM_HIP(hipMemcpyAsync(P->b.ents, T.ents.data(), T.ents.size() * sizeof(InjEnt), hipMemcpyHostToDevice, st));
        RTM_HIP(hipMemcpyAsync(P->b.cont, T.cont.data(), T.cont.size() * sizeof(Contrib), hipMemcpyHostToDevice, st));
    }
    RTM_HIP(hipMemcpyAsync(P->b.stasks, T.stasks.data(), T.stasks.size() * sizeof(SampleTask), hipMemcpyHostToDevice, st));
    RTM_HIP(hipMemcpyAsync(P->b.rnode, T.rnode.data(), T.rnode.size() * sizeof(int), hipMemcpyHostToDevice, st));
    RTM_HIP(hipMemcpyAsync(P->b.rw, T.rw.data(), T.rw.size() * sizeof(float), hipMemcpyHostToDevice, st));
    unsigned vr[2] = {0u, 0xffffffffu};
    const bool check = !(flags & RTM_F_SKIP_CHECK);
    if (check) {
        RTM_HIP(launch_vrange(v_pad, (int64_t)g.NX * g.NY * g.NZ, P->b.scal, st));
        RTM_HIP(hipMemcpyAsync(vr, P->b.scal, sizeof vr, hipMemcpyDeviceToHost, st));
    }
    RTM_HIP(hipStreamSynchronize(st));
    if (check) {
        float vmax, vmin;
        std::memcpy(&vmax, &vr[0], 4);
        std::memcpy(&vmin, &vr[1], 4);
        if (vr[0] >= 0x7f800000u || !(vmin > 0.f))
            return fail(RTM_ENUMERIC, "velocity must be finite and > 0 (max bits 0x%08x, min %g)", vr[0], (double)vmin);
        const double limit = std::sqrt(315.0 / (512.0 * g.ndim));
        const double courant = (double)vmax * dt / g.h;
        if (!(courant < limit))
            return fail(RTM_ECFL, "max(v) dt / h = %.6f >= stability limit %.6f", courant, limit);
    }
    return RTM_OK;
}

void fill_shot(const Prepared &P, ShotDev *S, const float *wavelet, const float *sig, float *rec_out, int nrec)
{
    std::memset(S, 0, sizeof *S);
    for (int i = 0; i < 4; ++i) S->fld[i] = P.b.fld[i];
    S->acc0 = P.b.acc0;
    S->acc1 = P.b.acc1;
    S->Dp = P.b.Dp;
    S->wav = wavelet;
    S->sig = sig;
    S->rec_out = rec_out;
    S->rnode = P.b.rnode;
    S->rw = P.b.rw;
    S->nrec = nrec;
    const GridInfo &g = P.g;
    S->ix0 = g.nb;
    S->ix1 = g.nb + (int)g.nx;
    S->iy0 = g.ndim == 3 ? g.nb : 0;
    S->iy1 = g.ndim == 3 ? g.nb + (int)g.ny : 1;
    S->iz0 = g.nb;
    S->iz1 = g.nb + (int)g.nz;
    S->L = g.L;
}

int upload_shot(const Prepared &P, const ShotDev &S)
{
    // The descriptor is small; it is copied from a host value that lives
    // until the call returns, after the stream synchronisation below.
    RTM_HIP(hipMemcpyAsync(P.b.shot, &S, sizeof S, hipMemcpyHostToDevice, P.st));
    RTM_HIP(hipStreamSynchronize(P.st));
    return RTM_OK;
}

int forward_loop(const Prepared &P, int nt, bool sample)
{
    const HostTables &T = P.T;
    const int ntiles = (int)T.tiles.size();
    const int nsample = sample ? (int)T.stasks.size() : 0;
    LoopTimer timer(sample ? kLoopModelFwd : kLoopRtmFwd, nt, P.st);
    for (int n = 0; n < nt; ++n)
        RTM_HIP(launch_fwd2d(P.tune.vec, P.b.shot, P.b.tiles, ntiles, T.nslots, P.b.ents, P.b.cont,
                             sample ? P.b.stasks : nullptr, nsample, n, P.st));
    timer.finish();
    return RTM_OK;
}

int zero_fields(const Prepared &P, int nf)
{
    for (int i = 0; i < nf; ++i) RTM_HIP(launch_fill(P.b.fld[i], P.g.L.total, 0.f, P.st));
    return RTM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int rtm_abi_version(void) { return RTM_ABI_VERSION; }

const char *rtm_last_error(void) { return t_err.c_str(); }

int rtm_set_tuning(int op, int vec, int zseg)
{
    if (vec != 1 && vec != 2 && vec != 4) return fail(RTM_EINVAL, "vec must be 1, 2 or 4");
    if (zseg < kMinZseg || zseg > 4096) return fail(RTM_EINVAL, "zseg must be in [%d, 4096]", kMinZseg);
    int packed = (vec << 16) | zseg;
    if (op == RTM_OP_MODEL) g_tune2d_fwd = packed;
    else if (op == RTM_OP_RTM || op == RTM_OP_VJP) g_tune2d_rev = packed;
    else return fail(RTM_EINVAL, "unknown op %d", op);
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
    if (op < RTM_OP_RBC_PAD || op > RTM_OP_VJP) return fail(RTM_EINVAL, "unknown op %d", op);
    if (op != RTM_OP_RBC_PAD && (nrec < 1 || nt < 1)) return fail(RTM_EINVAL, "nrec and nt must be >= 1");
    *bytes = carve(nullptr, g, op, nrec, nt).bytes;
    return RTM_OK;
}

int rtm_rbc_pad(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap, float *v_pad, void *ws,
                size_t ws_bytes, void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = grid_info(grid, &g);
    if (rc) return rc;
    if (!v_int || !v_pad) return fail(RTM_EINVAL, "v_int and v_pad must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    const unsigned *cap_bits = nullptr;
    if (!(v_cap > 0.f)) {
        size_t need = carve(nullptr, g, RTM_OP_RBC_PAD, 0, 0).bytes;
        if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
            return fail(RTM_EWORKSPACE, "v_cap <= 0 needs an aligned workspace of %zu bytes", need);
        unsigned *slot = carve(ws, g, RTM_OP_RBC_PAD, 0, 0).scal;
        RTM_HIP(launch_vmax(v_int, g.nx * g.ny * g.nz, slot, st));
        cap_bits = slot;
    }
    RTM_HIP(launch_rbc_pad(g.ndim, g.nb, g.nx, g.ny, g.nz, v_int, seed, v_cap, cap_bits, v_pad, st));
    return RTM_OK;
}

int rtm_pad_adjoint(const rtm_grid_t *grid, const float *v_int, uint64_t seed, float v_cap, const float *grad_v_pad,
                    float *grad_v_int, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    GridInfo g;
    int rc = grid_info(grid, &g);
    if (rc) return rc;
    if (!v_int || !grad_v_pad || !grad_v_int) return fail(RTM_EINVAL, "NULL array argument");
    hipStream_t st = (hipStream_t)stream;
    const unsigned *cap_bits = nullptr;
    if (!(v_cap > 0.f)) {
        size_t need = carve(nullptr, g, RTM_OP_RBC_PAD, 0, 0).bytes;
        if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
            return fail(RTM_EWORKSPACE, "v_cap <= 0 needs an aligned workspace of %zu bytes", need);
        unsigned *slot = carve(ws, g, RTM_OP_RBC_PAD, 0, 0).scal;
        RTM_HIP(launch_vmax(v_int, g.nx * g.ny * g.nz, slot, st));
        cap_bits = slot;
    }
    RTM_HIP(launch_pad_adjoint(g.ndim, g.nb, g.nx, g.ny, g.nz, v_int, seed, v_cap, cap_bits, grad_v_pad, grad_v_int,
                               st));
    return RTM_OK;
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
    Prepared P;
    rc = prepare(g, RTM_OP_MODEL, v_pad, dt, nt, src, nrec, rec, flags, ws, ws_bytes, stream, &P);
    if (rc) return rc;
    ShotDev S;
    fill_shot(P, &S, wavelet, nullptr, P.b.traces, nrec);
    hipStream_t st = P.st;
    RTM_HIP(launch_build_dp(g.L, v_pad, (float)(dt / g.h), P.b.Dp, st));
    if ((rc = zero_fields(P, 2))) return rc;
    if ((rc = upload_shot(P, S))) return rc;
    if ((rc = forward_loop(P, nt, true))) return rc;
    RTM_HIP(launch_sample(P.b.shot, P.b.stasks, (int)P.T.stasks.size(), nt, st));
    RTM_HIP(launch_transpose(P.b.traces, traces, nt + 1, nrec, st));
    if (p_last) RTM_HIP(launch_unpack(g.L, P.b.fld[nt & 1], p_last, st));
    if (p_prev) RTM_HIP(launch_unpack(g.L, P.b.fld[(nt + 1) & 1], p_prev, st));
    return RTM_OK;
}

static int reverse_common(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                          const float *src, int32_t nrec, const float *rec, const float *traces, bool grad,
                          int reinject, const rtm_probe_t *probe, uint32_t flags, void *ws, size_t ws_bytes,
                          void *stream, Prepared *P, bool want_wadj)
{
    GridInfo g;
    int rc = check_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, &g);
    if (rc) return rc;
    if (!traces) return fail(RTM_EINVAL, "traces is NULL");
    if (probe && probe->snap_k >= 0 && probe->snap_k > nt - 2)
        return fail(RTM_EINVAL, "probe step %d outside [0, nt - 2]", (int)probe->snap_k);
    rc = prepare(g, grad ? RTM_OP_VJP : RTM_OP_RTM, v_pad, dt, nt, src, nrec, rec, flags, ws, ws_bytes, stream, P);
    if (rc) return rc;
    ShotDev S;
    fill_shot(*P, &S, wavelet, P->b.traces, nullptr, nrec);
    hipStream_t st = P->st;
    RTM_HIP(launch_build_dp(g.L, v_pad, (float)(dt / g.h), P->b.Dp, st));
    if ((rc = zero_fields(*P, 4))) return rc;
    RTM_HIP(launch_fill(P->b.acc0, g.L.total, 0.f, st));
    if (!grad) RTM_HIP(launch_fill(P->b.acc1, g.L.total, 0.f, st));
    if (want_wadj) RTM_HIP(launch_fill(P->b.wadj, (int64_t)nt * kMaxNodes, 0.f, st));
    RTM_HIP(launch_transpose(traces, P->b.traces, nrec, nt + 1, st));
    if ((rc = upload_shot(*P, S))) return rc;
    // Forward pass: only the last two panels are kept (Algorithm 3).
    if ((rc = forward_loop(*P, nt, false))) return rc;
    // Receiver field start: mu^{nt} = D' h^2 R^T g^{nt}, mu^{nt+1} = 0.
    const HostTables &T = P->T;
    RTM_HIP(launch_inj_set(P->b.shot, 0, P->b.ents, T.nsrc_ent, T.nsrc_ent + T.nrec_ent, P->b.cont, nt, st));
    const int ntiles = (int)T.tiles.size();
    const bool probing = probe && probe->snap_k >= 0;
    // Probe copies would be timed with the loop: such calls are not recorded.
    LoopTimer timer(grad ? kLoopRevGrad : kLoopRevImage, nt, st, !probing);
    for (int k = nt - 1; k >= 0; --k) {
        RTM_HIP(launch_rev2d(P->tune.vec, grad, P->b.shot, P->b.tiles, ntiles, T.nslots, P->b.ents, P->b.cont, k,
                             reinject, want_wadj ? P->b.wadj : nullptr, st));
        if (probe && probe->snap_k >= 0) {
            if (k - 1 == probe->snap_k && probe->snap_p) RTM_HIP(launch_unpack(g.L, P->b.fld[(k - 1) & 1], probe->snap_p, st));
            if (k == probe->snap_k && probe->snap_mu) RTM_HIP(launch_unpack(g.L, P->b.fld[2 + (k & 1)], probe->snap_mu, st));
        }
    }
    timer.finish();
    return RTM_OK;
}

int rtm_rtm_shot(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                 const float *src, int32_t nrec, const float *rec, const float *traces, float eps_rel, float *image,
                 float *num, float *den, const rtm_probe_t *probe, uint32_t flags, void *ws, size_t ws_bytes,
                 void *stream)
{
    t_err.clear();
    if (!image) return fail(RTM_EINVAL, "image is NULL");
    if (!(eps_rel >= 0.f) || !std::isfinite(eps_rel)) return fail(RTM_EINVAL, "eps_rel must be finite and >= 0");
    Prepared P;
    int reinject = (flags & RTM_F_NO_REINJECT) ? 0 : 1;
    int rc = reverse_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, traces, false, reinject, probe, flags, ws,
                            ws_bytes, stream, &P, false);
    if (rc) return rc;
    RTM_HIP(launch_image(P.b.shot, 0, P.g.nx * P.g.ny * P.g.nz, P.b.scal, eps_rel, image, num, den, P.st));
    return RTM_OK;
}

int rtm_model_shot_vjp(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt, const float *wavelet,
                       const float *src, int32_t nrec, const float *rec, const float *grad_traces, float *grad_v_pad,
                       float *grad_wavelet, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    t_err.clear();
    if (!grad_v_pad) return fail(RTM_EINVAL, "grad_v_pad is NULL");
    Prepared P;
    int rc = reverse_common(grid, v_pad, dt, nt, wavelet, src, nrec, rec, grad_traces, true, 1, nullptr, flags, ws,
                            ws_bytes, stream, &P, grad_wavelet != nullptr);
    if (rc) return rc;
    const GridInfo &g = P.g;
    RTM_HIP(launch_grad(P.b.shot, 0, (int64_t)g.NX * g.NY * g.NZ, v_pad, (float)dt, grad_v_pad, P.st));
    if (grad_wavelet) RTM_HIP(launch_wadj(P.b.wadj, nt, (float)(1.0 / (g.h * g.h)), grad_wavelet, P.st));
    return RTM_OK;
}

}  // extern "C"
