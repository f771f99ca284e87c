// Host-logic check of librtm's runtime (tiles, injection tables, workspace
// layout, storage-RTM launch schedule) with the device launchers replaced by
// recorders: built with host AddressSanitizer / UBSan and run on the CPU by
// tests/test_host_logic.py.  No GPU call is made.
#include "api.hip"

#include <cstdio>
#include <map>
#include <set>
#include <tuple>

namespace rtm {
#include "stubs.inc"  // every other launcher: returns hipSuccess

// Storage schedule recorder: which field holds which p level, which levels
// are copied and which snapshot each reverse step images with.
struct Sim {
    const ShotDev *base = nullptr;
    std::vector<ShotDev> host;
    int nsh = 1;
    std::map<const float *, int> lev_of, mu_of;  // p and mu level held by each field
    std::vector<int> fsteps, rsteps;               // forward and reverse steps, in launch order
    std::map<int, int> sampled;                    // receiver samples recorded per level
    // a sample of level n from field `slot` of table T
    void sample(const ShotDev &T, int n, int slot)
    {
        if (lev_of.count(T.fld[slot]) == 0 || lev_of[T.fld[slot]] != n) ++errors;
        sampled[n]++;
    }
    float *snaps = nullptr;
    int64_t ncell = 0;
    int stride = 1, phase = 0, last_k = 1 << 30;
    std::map<int, int> stored, used;
    long errors = 0;
    const ShotDev &tab(const ShotDev *p)
    {
        const size_t i = (size_t)(p - base);
        if (i != 0 && i != (size_t)nsh) ++errors;
        return host[i < host.size() ? i : 0];
    }
    const ShotDev &other(const ShotDev *p) { return host[(p - base) == 0 ? nsh : 0]; }
} SIM;

hipError_t launch_fwd2d(int, int, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *, const Contrib *,
                        const SampleTask *stasks, int nsample, int n, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    if (SIM.lev_of[T.fld[n & 1]] != n) ++SIM.errors;
    if (stasks && nsample > 0) SIM.sample(T, n, n & 1);
    SIM.lev_of[T.fld[(n + 1) & 1]] = n + 1;
    SIM.fsteps.push_back(n);
    return hipSuccess;
}
hipError_t launch_fwd3d(int, int, const ShotDev *shots, const Tile3D *, int, int, const InjEnt *, const Contrib *,
                        const SampleTask *stasks, int nsample, int n, hipStream_t)
{
    return launch_fwd2d(0, 0, shots, nullptr, 0, 0, nullptr, nullptr, stasks, nsample, n, nullptr);
}
hipError_t launch_fwd2d_t2(int, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *, const Contrib *,
                           const SampleTask *stasks, int nsample, int n, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    if (SIM.lev_of[T.fld[n & 1]] != n) ++SIM.errors;
    if (stasks && nsample > 0) {
        if (n > 0) SIM.sample(T, n - 1, (n - 1) & 1);
        SIM.sample(T, n, n & 1);
    }
    const ShotDev &U = SIM.other(shots);
    SIM.lev_of[U.fld[(n + 1) & 1]] = n + 1;
    SIM.lev_of[U.fld[(n + 2) & 1]] = n + 2;
    SIM.fsteps.push_back(n);
    SIM.fsteps.push_back(n + 1);
    return hipSuccess;
}
hipError_t launch_fwd2d_t3(int, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *, const Contrib *,
                           const SampleTask *stasks, int nsample, int n, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    if (SIM.lev_of[T.fld[n & 1]] != n || SIM.lev_of[T.fld[(n + 1) & 1]] != n - 1) ++SIM.errors;
    if (stasks && nsample > 0) {
        if (n >= 3) SIM.sample(T, n - 2, 6);
        if (n >= 1) SIM.sample(T, n - 1, (n - 1) & 1);
        SIM.sample(T, n, n & 1);
        if (!T.fld[2] || !T.fld[6] || T.sz1 <= T.sz0) ++SIM.errors;
        SIM.lev_of[T.fld[2]] = n + 1;  // the middle level, on the receiver rows
    }
    SIM.lev_of[T.fld[4 + (n & 1)]] = n + 2;
    SIM.lev_of[T.fld[4 + ((n + 1) & 1)]] = n + 3;
    for (int i = 0; i < 3; ++i) SIM.fsteps.push_back(n + i);
    return hipSuccess;
}
hipError_t launch_sample(const ShotDev *shots, const SampleTask *, int ntask, int n, int slot, hipStream_t)
{
    if (ntask > 0) SIM.sample(SIM.tab(shots), n, slot);
    return hipSuccess;
}
hipError_t launch_inj_set(const ShotDev *shots, const InjEnt *, int, int, const Contrib *, int step, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    SIM.mu_of[T.fld[2 + (step & 1)]] = step;
    SIM.mu_of[T.fld[2 + ((step + 1) & 1)]] = step + 1;  // zero: cleared with the job's fields
    return hipSuccess;
}
// Reverse steps read p^k, p^{k+1}, mu^{k+1}, mu^{k+2} from the current set.
static void rev_reads(const ShotDev &T, int k)
{
    if (SIM.lev_of[T.fld[k & 1]] != k || SIM.lev_of[T.fld[(k + 1) & 1]] != k + 1) ++SIM.errors;
    if (SIM.mu_of[T.fld[2 + ((k + 1) & 1)]] != k + 1 || SIM.mu_of[T.fld[2 + (k & 1)]] != k + 2) ++SIM.errors;
}
hipError_t launch_rev2d(int, int, bool, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *,
                        const Contrib *, int k, int, float *, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    rev_reads(T, k);
    SIM.lev_of[T.fld[(k + 1) & 1]] = k - 1;
    SIM.mu_of[T.fld[2 + (k & 1)]] = k;
    SIM.rsteps.push_back(k);
    return hipSuccess;
}
hipError_t launch_rev2d_t2(int, bool, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *,
                           const Contrib *, int k, int, float *, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    rev_reads(T, k);
    SIM.lev_of[T.fld[4 + ((k + 1) & 1)]] = k - 1;
    SIM.lev_of[T.fld[4 + (k & 1)]] = k - 2;
    SIM.mu_of[T.fld[6 + (k & 1)]] = k;
    SIM.mu_of[T.fld[6 + ((k + 1) & 1)]] = k - 1;
    SIM.rsteps.push_back(k);
    SIM.rsteps.push_back(k - 1);
    return hipSuccess;
}
hipError_t launch_rev2d_t3(int, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *, const Contrib *,
                           int k, int, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    rev_reads(T, k);
    SIM.lev_of[T.fld[4 + (k & 1)]] = k - 2;
    SIM.lev_of[T.fld[4 + ((k + 1) & 1)]] = k - 3;
    SIM.mu_of[T.fld[6 + ((k + 1) & 1)]] = k - 1;
    SIM.mu_of[T.fld[6 + (k & 1)]] = k - 2;
    for (int i = 0; i < 3; ++i) SIM.rsteps.push_back(k - i);
    return hipSuccess;
}
hipError_t launch_snap_store(const ShotDev *shots, int shot, int lev, int64_t ninterior, float *out, hipStream_t)
{
    const ShotDev &T = SIM.tab(shots);
    const int64_t off = out - SIM.snaps;
    if (shot != 0 || ninterior != SIM.ncell || off % SIM.ncell) ++SIM.errors;
    const int m = SIM.phase + (int)(off / SIM.ncell) * SIM.stride;
    if (SIM.lev_of[T.fld[lev]] != m) ++SIM.errors;
    SIM.stored[m]++;
    return hipSuccess;
}
hipError_t launch_recv2d(int, int, const ShotDev *shots, const Tile2D *, int, int, const InjEnt *, const Contrib *,
                         int k, const float *snap, hipStream_t)
{
    SIM.tab(shots);
    if (SIM.last_k != (1 << 30) && k != SIM.last_k - 1) ++SIM.errors;
    SIM.last_k = k;
    const bool st = k >= SIM.phase && (k - SIM.phase) % SIM.stride == 0;
    const float *want = st ? SIM.snaps + (int64_t)((k - SIM.phase) / SIM.stride) * SIM.ncell : nullptr;
    if (snap != want) ++SIM.errors;
    if (st) SIM.used[k]++;
    return hipSuccess;
}
hipError_t launch_recv3d(int, int, const ShotDev *shots, const Tile3D *, int, int, const InjEnt *, const Contrib *,
                         int k, const float *snap, hipStream_t st)
{
    return launch_recv2d(0, 0, shots, nullptr, 0, 0, nullptr, nullptr, k, snap, st);
}
}  // namespace rtm

static long g_bad = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            if (g_bad++ < 20) {               \
                std::printf(__VA_ARGS__);     \
                std::printf("\n");             \
            }                                 \
        }                                     \
    } while (0)

// Every entry of a tile's own lists lies in the cells the tile owns and
// appears once; every first-step entry of a tile of S > 1 steps lies in its
// strip span and rows [z0 - 4 (S - 1), z1 + 4 (S - 1)), every second-step
// entry (S = 3) in the span and rows [z0 - 4, z1 + 4), sorted by row; and
// every node lies in the first- and second-step lists of each tile whose
// regions contain it.
static void check_entries(const Job &J, const Tiling &T, const char *name)
{
    const int span = 64 * T.tune.vec;
    const int off = T.ndim == 2 && T.steps > 1 ? 4 * (T.steps - 1) : 0;
    std::set<std::tuple<int, int, int, int, int>> listed;  // (tile, kind, z, y, x)
    for (int t = 0; t < T.count(); ++t) {
        auto lists = [&](int b, int e, int kind) {
            std::set<std::tuple<int, int, int>> seen;
            for (int i = b; i < e; ++i) {
                CHECK(i >= 0 && i < (int)T.ents.size(), "%s: entry index out of range", name);
                const InjEnt &E = T.ents[i];
                CHECK(seen.insert(std::make_tuple(E.z, E.y, E.x)).second, "%s tile %d: duplicate node", name, t);
                const GridInfo &g = J.shots[E.shot].g;
                bool own;
                if (T.ndim == 3) {
                    const Tile3D &tl = T.tiles3[t];
                    own = E.x >= tl.x0 && E.x < tl.x0 + span && E.y >= tl.y0 && E.y < tl.y0 + T.tune.ty &&
                          E.z >= tl.z0 && E.z < tl.z1 && E.x < g.NX && E.y < g.NY;
                } else {
                    const Tile2D &tl = T.tiles[t];
                    const int ext = kind >= 4 ? 4 : off;
                    if (kind >= 2)
                        own = off > 0 && (kind < 4 || T.steps == 3) && E.x >= tl.x0 && E.x < tl.x0 + span &&
                              E.z >= tl.z0 - ext && E.z < tl.z1 + ext;
                    else if (off > 0)
                        own = E.x >= tl.x0 + off && E.x < tl.x0 + span - off && E.z >= tl.z0 && E.z < tl.z1 &&
                              E.x < g.NX;
                    else
                        own = E.x >= tl.x0 && E.x < tl.x0 + span * T.tune.tx && E.z >= tl.z0 && E.z < tl.z1 &&
                              E.x < g.NX;
                    if (kind >= 2 && i > b) CHECK(T.ents[i - 1].z <= E.z, "%s: step list unsorted", name);
                    listed.insert(std::make_tuple(t, kind, E.z, E.y, E.x));
                }
                CHECK(own, "%s tile %d kind %d: node (%d,%d,%d) not in the tile", name, t, kind, E.z, E.y, E.x);
                CHECK(E.cbeg >= 0 && E.cend <= (int)T.cont.size() && E.cbeg < E.cend, "%s: bad contributions", name);
            }
        };
        if (T.ndim == 3) {
            const Tile3D &tl = T.tiles3[t];
            lists(tl.sbeg, tl.send, 0);
            lists(tl.rbeg, tl.rend, 1);
        } else {
            const Tile2D &tl = T.tiles[t];
            lists(tl.sbeg, tl.send, 0);
            lists(tl.rbeg, tl.rend, 1);
            lists(tl.s1beg, tl.s1end, 2);
            lists(tl.r1beg, tl.r1end, 3);
            lists(tl.s2beg, tl.s2end, 4);
            lists(tl.r2beg, tl.r2end, 5);
        }
    }
    if (off == 0) return;
    // completeness: each owned node, in every tile of its shot whose step
    // regions contain it
    for (int t = 0; t < T.count(); ++t) {
        const Tile2D &tl = T.tiles[t];
        for (int kind = 0; kind < 2; ++kind)
            for (int i = kind == 0 ? tl.sbeg : tl.rbeg; i < (kind == 0 ? tl.send : tl.rend); ++i) {
                const InjEnt &E = T.ents[i];
                for (int u = 0; u < T.count(); ++u) {
                    const Tile2D &o = T.tiles[u];
                    if (o.shot != tl.shot || E.x < o.x0 || E.x >= o.x0 + span) continue;
                    if (E.z >= o.z0 - off && E.z < o.z1 + off)
                        CHECK(listed.count(std::make_tuple(u, kind + 2, E.z, E.y, E.x)),
                              "%s: node (%d,%d) missing from tile %d's first-step list", name, E.z, E.x, u);
                    if (T.steps == 3 && E.z >= o.z0 - 4 && E.z < o.z1 + 4)
                        CHECK(listed.count(std::make_tuple(u, kind + 4, E.z, E.y, E.x)),
                              "%s: node (%d,%d) missing from tile %d's second-step list", name, E.z, E.x, u);
                }
            }
    }
}

// Each table uploaded into the workspace fits the region the layout gave it
// (the layout is sized from position-independent bounds).
static void check_layout(const Job &J, const char *name)
{
    const WsLayout &w = J.ws;
    auto fits = [&](const char *what, size_t off, size_t n, size_t next) {
        CHECK(n == 0 || off + n <= next, "%s: %s overflows its region (%zu + %zu > %zu)", name, what, off, n, next);
    };
    const size_t tb = kTileBytes;
    fits("shots", w.shots, sizeof(ShotDev) * 2 * J.shots.size(), w.tiles_f);
    fits("tiles_f", w.tiles_f, tb * J.fw.count(), w.ents_f);
    fits("ents_f", w.ents_f, sizeof(InjEnt) * J.fw.ents.size(), w.cont_f);
    fits("cont_f", w.cont_f, sizeof(Contrib) * J.fw.cont.size(), w.tiles_r);
    fits("tiles_r", w.tiles_r, tb * J.rv.count(), w.ents_r);
    fits("ents_r", w.ents_r, sizeof(InjEnt) * J.rv.ents.size(), w.cont_r);
    fits("cont_r", w.cont_r, sizeof(Contrib) * J.rv.cont.size(), w.tiles_f2);
    fits("tiles_f2", w.tiles_f2, tb * J.fw2.count(), w.ents_f2);
    fits("ents_f2", w.ents_f2, sizeof(InjEnt) * J.fw2.ents.size(), w.cont_f2);
    fits("cont_f2", w.cont_f2, sizeof(Contrib) * J.fw2.cont.size(), w.tiles_r2);
    fits("tiles_r2", w.tiles_r2, tb * J.rv2.count(), w.ents_r2);
    fits("ents_r2", w.ents_r2, sizeof(InjEnt) * J.rv2.ents.size(), w.cont_r2);
    fits("cont_r2", w.cont_r2, sizeof(Contrib) * J.rv2.cont.size(), w.stasks);
    CHECK(w.bytes <= single_bytes(J.shots[0].g, J.op, J.shots[0].nrec, J.nt), "%s: layout larger than advertised", name);
}

static std::vector<float> receivers(int ndim, int nx, int ny)
{
    std::vector<float> rec;
    for (int i = 0; i < nx - 1; ++i)
        for (int y = 0; y < (ndim == 3 ? ny : 1); y += 2) {
            rec.push_back((float)i + (i % 3 == 0 ? 0.25f : 0.f));
            rec.push_back((float)y);
            rec.push_back(i % 2 ? 2.0f : 2.5f);
        }
    return rec;
}

static int tables(int ndim, int vec, int tx, int ty, int zseg, int steps)
{
    rtm_grid_t gr{ndim, 7, ndim == 2 ? 301 : 70, ndim == 3 ? 33 : 1, 41, 10.0};
    GridInfo g;
    if (grid_info(&gr, &g)) return 1;
    rtm_set_tuning(RTM_TUNE_EXACT, 1, 0);
    if (ndim == 2) {
        rtm_set_tuning2d(RTM_OP_MODEL, vec, tx, zseg);
        rtm_set_tuning2d(RTM_OP_RTM, vec, tx, zseg);
        rtm_set_steps_per_launch(RTM_OP_MODEL, steps);
        rtm_set_steps_per_launch(RTM_OP_RTM, steps);
    } else {
        rtm_set_tuning3d(RTM_OP_MODEL, vec, ty, zseg);
        rtm_set_tuning3d(RTM_OP_RTM, vec, ty, zseg);
    }
    float src[3] = {ndim == 2 ? 150.3f : 33.3f, ndim == 3 ? 11.5f : 0.f, 3.7f};
    std::vector<float> rec = receivers(ndim, (int)gr.nx, (int)gr.ny);
    for (int op : {RTM_OP_MODEL, RTM_OP_RTM, RTM_OP_STORAGE, RTM_OP_VJP}) {
        Job J;
        std::vector<float> fake(1);
        int rc = single_job(J, op, g, fake.data(), 1e-3, 20, fake.data(), src, (int)rec.size() / 3, rec.data(), 0);
        CHECK(rc == 0, "single_job failed: %s", t_err.c_str());
        if (rc) continue;
        check_entries(J, J.fw, "fw");
        check_entries(J, J.rv, "rv");
        check_entries(J, J.fw2, "fw2");
        check_entries(J, J.rv2, "rv2");
        check_layout(J, "layout");
    }
    rtm_set_tuning(RTM_TUNE_EXACT, 0, 0);
    return 0;
}

static void storage_schedule(int ndim, int nt, int stride, int phase, int steps)
{
    rtm_grid_t gr{ndim, 6, 40, ndim == 3 ? 20 : 1, 23, 10.0};
    GridInfo g;
    grid_info(&gr, &g);
    rtm_set_steps_per_launch(RTM_OP_MODEL, steps);
    float src[3] = {17.3f, ndim == 3 ? 9.0f : 0.f, 3.7f};
    std::vector<float> rec;
    for (int i = 0; i < 10; ++i) {
        rec.push_back(0.5f + 3.7f * i);
        rec.push_back(ndim == 3 ? 5.f : 0.f);
        rec.push_back(2.25f);
    }
    Job J;
    std::vector<float> fake(1);
    if (single_job(J, RTM_OP_STORAGE, g, fake.data(), 1e-3, nt, fake.data(), src, 10, rec.data(), 0)) {
        CHECK(false, "storage single_job failed: %s", t_err.c_str());
        return;
    }
    std::vector<char> ws(J.ws.bytes + 256);
    Dev D{(char *)(((uintptr_t)ws.data() + 255) & ~(uintptr_t)255)};
    int64_t count = 0;
    rtm_storage_count(nt, stride, phase, &count);
    SIM = Sim();
    SIM.ncell = g.nx * g.ny * g.nz;
    std::vector<float> snaps((size_t)std::max<int64_t>(1, count * SIM.ncell));
    SIM.snaps = snaps.data();
    SIM.stride = stride;
    SIM.phase = phase;
    ShotIn &S = J.shots[0];
    S.snaps = snaps.data();
    S.stride = stride;
    S.phase = phase;
    fill_shot_devs(J, D, SIM.host);
    SIM.base = D.at<ShotDev>(J.ws.shots);
    SIM.lev_of[SIM.host[0].fld[0]] = 0;
    SIM.lev_of[SIM.host[0].fld[1]] = -1;
    const int rc = job_launch(J, D, nullptr, nullptr, false);
    CHECK(rc == 0, "job_launch failed: %s", t_err.c_str());
    for (int k = 0; k < nt; ++k) {
        const int want = (k >= phase && (k - phase) % stride == 0) ? 1 : 0;
        CHECK(SIM.stored[k] == want && SIM.used[k] == want, "storage nt %d stride %d phase %d steps %d: level %d "
              "stored %d used %d", nt, stride, phase, steps, k, SIM.stored[k], SIM.used[k]);
    }
    CHECK(SIM.errors == 0, "storage nt %d stride %d phase %d steps %d: %ld schedule errors", nt, stride, phase, steps,
          SIM.errors);
}

// RTM launch schedule for S steps per launch: the forward launches take
// steps 0 .. nt - 1 in order, each reading the levels it needs; the reverse
// launches take steps nt - 1 .. 0 in order, each reading p^k, p^{k+1},
// mu^{k+1}, mu^{k+2} from where the previous launches left them.  Modeling:
// the same forward order, and every level 0 .. nt recorded exactly once
// from the field (or middle-level buffer) holding it.
static void rtm_schedule(int nt, int steps)
{
    rtm_grid_t gr{2, 6, 40, 1, 23, 10.0};
    GridInfo g;
    grid_info(&gr, &g);
    rtm_set_tuning(RTM_TUNE_EXACT, 1, 0);  // small jobs would otherwise be narrowed to two steps
    rtm_set_steps_per_launch(RTM_OP_MODEL, steps);
    rtm_set_steps_per_launch(RTM_OP_RTM, steps);
    float src[3] = {17.3f, 0.f, 3.7f};
    std::vector<float> rec;
    for (int i = 0; i < 10; ++i) {
        rec.push_back(0.5f + 3.7f * i);
        rec.push_back(0.f);
        rec.push_back(2.25f);
    }
    Job J;
    std::vector<float> fake(1);
    if (single_job(J, RTM_OP_RTM, g, fake.data(), 1e-3, nt, fake.data(), src, 10, rec.data(), 0)) {
        CHECK(false, "rtm single_job failed: %s", t_err.c_str());
        return;
    }
    std::vector<char> ws(J.ws.bytes + 256);
    Dev D{(char *)(((uintptr_t)ws.data() + 255) & ~(uintptr_t)255)};
    SIM = Sim();
    fill_shot_devs(J, D, SIM.host);
    SIM.base = D.at<ShotDev>(J.ws.shots);
    SIM.lev_of[SIM.host[0].fld[0]] = 0;
    SIM.lev_of[SIM.host[0].fld[1]] = -1;
    const int rc = job_launch(J, D, nullptr, nullptr, false);
    CHECK(rc == 0, "job_launch failed: %s", t_err.c_str());
    bool ok = (int)SIM.fsteps.size() == nt && (int)SIM.rsteps.size() == nt;
    for (int i = 0; ok && i < nt; ++i) ok = SIM.fsteps[i] == i && SIM.rsteps[i] == nt - 1 - i;
    CHECK(ok, "rtm nt %d steps %d: forward %zu / reverse %zu steps out of order", nt, steps, SIM.fsteps.size(),
          SIM.rsteps.size());
    CHECK(SIM.errors == 0, "rtm nt %d steps %d: %ld schedule errors", nt, steps, SIM.errors);
    // gradient (two steps per launch at most): the same reverse order
    Job V;
    if (single_job(V, RTM_OP_VJP, g, fake.data(), 1e-3, nt, fake.data(), src, 10, rec.data(), 0)) {
        CHECK(false, "vjp single_job failed: %s", t_err.c_str());
        return;
    }
    std::vector<char> wv(V.ws.bytes + 256);
    Dev DV{(char *)(((uintptr_t)wv.data() + 255) & ~(uintptr_t)255)};
    SIM = Sim();
    fill_shot_devs(V, DV, SIM.host);
    SIM.base = DV.at<ShotDev>(V.ws.shots);
    SIM.lev_of[SIM.host[0].fld[0]] = 0;
    SIM.lev_of[SIM.host[0].fld[1]] = -1;
    CHECK(job_launch(V, DV, nullptr, nullptr, false) == 0, "vjp job_launch failed: %s", t_err.c_str());
    bool vok = (int)SIM.rsteps.size() == nt;
    for (int i = 0; vok && i < nt; ++i) vok = SIM.rsteps[i] == nt - 1 - i;
    CHECK(vok && SIM.errors == 0 && V.rv2.steps == (steps > 1 ? 2 : 1),
          "vjp nt %d steps %d: reverse steps out of order or %ld schedule errors", nt, steps, SIM.errors);
    check_layout(V, "vjp layout");
    // modeling: every level 0 .. nt recorded once, from the field holding it
    Job M;
    if (single_job(M, RTM_OP_MODEL, g, fake.data(), 1e-3, nt, fake.data(), src, 10, rec.data(), 0)) {
        CHECK(false, "model single_job failed: %s", t_err.c_str());
        return;
    }
    std::vector<char> wm(M.ws.bytes + 256);
    Dev DM{(char *)(((uintptr_t)wm.data() + 255) & ~(uintptr_t)255)};
    SIM = Sim();
    fill_shot_devs(M, DM, SIM.host);
    SIM.base = DM.at<ShotDev>(M.ws.shots);
    SIM.lev_of[SIM.host[0].fld[0]] = 0;
    SIM.lev_of[SIM.host[0].fld[1]] = -1;
    CHECK(job_launch(M, DM, nullptr, nullptr, false) == 0, "model job_launch failed: %s", t_err.c_str());
    bool all = (int)SIM.fsteps.size() == nt;
    for (int i = 0; all && i < nt; ++i) all = SIM.fsteps[i] == i;
    for (int k = 0; k <= nt; ++k) all = all && SIM.sampled[k] == 1;
    CHECK(all && (int)SIM.sampled.size() == nt + 1, "model nt %d steps %d: levels not each recorded once", nt,
          steps);
    CHECK(SIM.errors == 0, "model nt %d steps %d: %ld schedule errors", nt, steps, SIM.errors);
    CHECK(M.fw2.steps == (steps > 1 ? steps : 1) && J.rv2.steps == (steps > 1 ? steps : 1),
          "nt %d: tilings of %d / %d steps, %d asked", nt, M.fw2.steps, J.rv2.steps, steps);
    rtm_set_steps_per_launch(RTM_OP_RTM, 2);
    rtm_set_tuning(RTM_TUNE_EXACT, 0, 0);
}

int main()
{
    int cases = 0;
    for (int vec : {1, 2, 4})
        for (int tx : {1, 2, 4})
            for (int steps : {1, 2, 3}) {
                tables(2, vec, tx, 1, steps > 1 ? 9 : 18, steps);
                ++cases;
            }
    tables(2, 4, 1, 1, 108, 2);
    tables(2, 4, 1, 1, 108, 3);
    for (int steps : {1, 2, 3})
        for (int nt : {1, 2, 3, 4, 5, 6, 7, 20}) {
            rtm_schedule(nt, steps);
            ++cases;
        }
    for (int vec : {1, 2})
        for (int ty : {4, 8}) {
            tables(3, vec, 1, ty, 18, 1);
            ++cases;
        }
    for (int steps : {1, 2, 3})
        for (int nt : {1, 2, 7, 8, 31})
            for (auto sp : {std::make_pair(1, 0), std::make_pair(3, 2), std::make_pair(10, 9), std::make_pair(4, 1)}) {
                storage_schedule(2, nt, sp.first, sp.second, steps);
                ++cases;
            }
    for (int nt : {5, 12}) storage_schedule(3, nt, 3, 1, 1);
    rtm_set_steps_per_launch(RTM_OP_MODEL, 2);
    std::printf("%d cases, %ld problems\n", cases, g_bad);
    if (g_bad == 0) std::printf("ALL OK\n");
    return g_bad ? 1 : 0;
}
