// 3-D propagation kernels for gfx950.
//
// A workgroup of TY wavefronts owns a tile of 64 * VEC x cells by TY rows in
// y and marches down z over [z0, z1) (a multiple of the 9-plane register
// queue).  Wavefront w holds row y0 + w:
//  - z-neighbours come from its register queue of planes z-4 .. z+4;
//  - x-neighbours from the adjacent lanes through DPP (plus the 4-cell strip
//    halo from one extra load by lanes 0 and 63);
//  - y-neighbours from an LDS copy of the centre plane z: every wavefront
//    writes its row there and the first ones load the 4 + 4 halo rows of the
//    tile.  The copy is double-buffered, so one barrier per plane suffices.
// Stencil, update and injection follow the 2-D kernels (difference form that
// is exactly zero on constant fields; source and receiver terms added after
// the march by the lanes that stored the cells).
#include "stencil.h"

namespace rtm {
namespace {

template <int VEC, int TY>
struct Lds {
    float row[2][TY + 8][64 * VEC];
};

// Number of y-halo rows a wave loads per plane (8 halo rows over TY waves).
template <int TY>
constexpr int halo_per_wave() { return (8 + TY - 1) / TY; }

// Everything one field needs from memory for one plane of one row, loaded
// one plane ahead (software pipelining across the per-plane barrier).
template <int VEC, int TY>
struct FieldNext {
    float q[VEC];                         // row z + 4 of the register queue
    float halo[halo_per_wave<TY>()][VEC];  // this wave's y-halo rows of plane z
    f4v hv;                               // strip-end x-halo (lanes 0 and 63)
};

template <int VEC>
struct Ctx3 {
    int64_t pitch, plane;
    int x, x0, y, y0, NX, NY, lane, w;
    bool liveX, live, own, rowlive;
};

// Issues the loads of field f for plane z (queue row z + 4, y-halo rows and
// x-halo of plane z).
template <int VEC, int TY>
__device__ __forceinline__ void field_prefetch(const Ctx3<VEC> &C, const gfloat *f, int z, FieldNext<VEC, TY> &nx)
{
    const gfloat *pz = f + (int64_t)z * C.plane;
#pragma unroll
    for (int j = 0; j < VEC; ++j) nx.q[j] = 0.f;
    if (C.live) ldv<VEC>(pz + 4 * C.plane + (int64_t)C.y * C.pitch + C.x, nx.q);
#pragma unroll
    for (int i = 0; i < halo_per_wave<TY>(); ++i) {
        const int h = C.w + i * TY;
#pragma unroll
        for (int j = 0; j < VEC; ++j) nx.halo[i][j] = 0.f;
        if (h < 8) {
            const int yh = h < 4 ? C.y0 - 4 + h : C.y0 + TY + (h - 4);
            if (C.liveX && yh < C.NY + kRadius) ldv<VEC>(pz + (int64_t)yh * C.pitch + C.x, nx.halo[i]);
        }
    }
    const int xr = C.x0 + 64 * VEC;
    const bool left = C.rowlive && C.lane == 0, right = C.rowlive && C.lane == 63 && xr < C.NX + kRadius;
    nx.hv = f4v{0.f, 0.f, 0.f, 0.f};
    if (left || right) nx.hv = *(const gf4v *)(pz + (int64_t)C.y * C.pitch + (left ? C.x0 - 4 : xr));
}

// Writes the centre row (queue slot of plane z) and the y-halo rows into
// LDS buffer `buf`; returns the x-halo split into left / right.
template <int VEC, int TY>
__device__ __forceinline__ void field_publish(const Ctx3<VEC> &C, Lds<VEC, TY> &L, int buf, const float (&c)[VEC],
                                              const FieldNext<VEC, TY> &nx, float (&hl)[4], float (&hr)[4])
{
#pragma unroll
    for (int j = 0; j < VEC; ++j) L.row[buf][4 + C.w][C.lane * VEC + j] = c[j];
#pragma unroll
    for (int i = 0; i < halo_per_wave<TY>(); ++i) {
        const int h = C.w + i * TY;
        if (h < 8) {
            const int slot = h < 4 ? h : TY + 4 + (h - 4);
#pragma unroll
            for (int j = 0; j < VEC; ++j) L.row[buf][slot][C.lane * VEC + j] = nx.halo[i][j];
        }
    }
    const bool left = C.lane == 0, right = C.lane == 63;
    hl[0] = left ? nx.hv.x : 0.f; hl[1] = left ? nx.hv.y : 0.f; hl[2] = left ? nx.hv.z : 0.f; hl[3] = left ? nx.hv.w : 0.f;
    hr[0] = right ? nx.hv.x : 0.f; hr[1] = right ? nx.hv.y : 0.f; hr[2] = right ? nx.hv.z : 0.f; hr[3] = right ? nx.hv.w : 0.f;
}

// Unscaled 3-D Laplacian of the centre cells of this wave.
template <int VEC, int TY>
__device__ __forceinline__ void lap3(const Lds<VEC, TY> &L, int buf, int w, int lane, const float (&ext)[VEC + 8],
                                     const float (&qa)[VEC], const float (&qb)[VEC], const float (&qc)[VEC],
                                     const float (&qd)[VEC], const float (&qe)[VEC], const float (&qf)[VEC],
                                     const float (&qg)[VEC], const float (&qh)[VEC], const float (&qi)[VEC],
                                     float (&lap)[VEC])
{
    // qa..qi: planes z-4 .. z+4 (qe is the centre).
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const int col = lane * VEC + j;
        const float c = qe[j], c2 = c + c;
        float l = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        l += d2(c2, L.row[buf][3 + w][col], L.row[buf][5 + w][col], L.row[buf][2 + w][col], L.row[buf][6 + w][col],
                L.row[buf][1 + w][col], L.row[buf][7 + w][col], L.row[buf][w][col], L.row[buf][8 + w][col]);
        l += d2(c2, qd[j], qf[j], qc[j], qg[j], qb[j], qh[j], qa[j], qi[j]);
        lap[j] = l;
    }
}

template <int VEC>
__device__ __forceinline__ void plane_prefetch(const Ctx3<VEC> &C, const gfloat *f, int z, float (&v)[VEC])
{
#pragma unroll
    for (int j = 0; j < VEC; ++j) v[j] = 0.f;
    if (C.live) ldv<VEC>(f + (int64_t)z * C.plane + (int64_t)C.y * C.pitch + C.x, v);
}

template <int VEC, int TY, int S>
__device__ __forceinline__ void fwd3_plane(const Ctx3<VEC> &C, Lds<VEC, TY> &L, const gfloat *pc, gfloat *po,
                                           const gfloat *Dp, float (&q)[9][VEC], FieldNext<VEC, TY> &nx,
                                           float (&nold)[VEC], float (&nd)[VEC], int z, int z0, int z1)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int buf = (z - z0) & 1;
    float old[VEC], d[VEC], hl[4], hr[4];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        q[r8][j] = nx.q[j];
        old[j] = nold[j];
        d[j] = nd[j];
    }
    field_publish<VEC, TY>(C, L, buf, q[r4], nx, hl, hr);
    if (z + 1 < z1) {
        field_prefetch<VEC, TY>(C, pc, z + 1, nx);
        plane_prefetch<VEC>(C, po, z + 1, nold);
        plane_prefetch<VEC>(C, Dp, z + 1, nd);
    }
    float ext[VEC + 8];
    exchange_row<VEC>(q[r4], hl, hr, ext);
    __syncthreads();
    float lap[VEC], out[VEC];
    lap3<VEC, TY>(L, buf, C.w, C.lane, ext, q[r0], q[r1], q[r2], q[r3], q[r4], q[r5], q[r6], q[r7], q[r8], lap);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q[r4][j];
        out[j] = fmaf(d[j], lap[j], (c + c) - old[j]);
    }
    if (C.own) stv<VEC>(po + (int64_t)z * C.plane + (int64_t)C.y * C.pitch + C.x, out);
}

template <int VEC, int TY, bool GRAD, int S>
__device__ __forceinline__ void rev3_plane(const Ctx3<VEC> &C, Lds<VEC, TY> &LP, Lds<VEC, TY> &LM,
                                           const gfloat *P0, gfloat *P1, const gfloat *M0, gfloat *M1,
                                           const gfloat *Dp, gfloat *A0, gfloat *A1, float (&qp)[9][VEC],
                                           float (&qm)[9][VEC], FieldNext<VEC, TY> &np_, FieldNext<VEC, TY> &nm_,
                                           float (&np1)[VEC], float (&nm1)[VEC], float (&nd)[VEC], int z, int z0,
                                           int z1, bool img_row)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int buf = (z - z0) & 1;
    float p1[VEC], m1[VEC], d[VEC], hlp[4], hrp[4], hlm[4], hrm[4];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        qp[r8][j] = np_.q[j];
        qm[r8][j] = nm_.q[j];
        p1[j] = np1[j];
        m1[j] = nm1[j];
        d[j] = nd[j];
    }
    field_publish<VEC, TY>(C, LP, buf, qp[r4], np_, hlp, hrp);
    field_publish<VEC, TY>(C, LM, buf, qm[r4], nm_, hlm, hrm);
    if (z + 1 < z1) {
        field_prefetch<VEC, TY>(C, P0, z + 1, np_);
        field_prefetch<VEC, TY>(C, M0, z + 1, nm_);
        plane_prefetch<VEC>(C, P1, z + 1, np1);
        plane_prefetch<VEC>(C, M1, z + 1, nm1);
        plane_prefetch<VEC>(C, Dp, z + 1, nd);
    }
    float extp[VEC + 8], extm[VEC + 8];
    exchange_row<VEC>(qp[r4], hlp, hrp, extp);
    exchange_row<VEC>(qm[r4], hlm, hrm, extm);
    __syncthreads();
    float lp[VEC], lm[VEC];
    lap3<VEC, TY>(LP, buf, C.w, C.lane, extp, qp[r0], qp[r1], qp[r2], qp[r3], qp[r4], qp[r5], qp[r6], qp[r7], qp[r8], lp);
    lap3<VEC, TY>(LM, buf, C.w, C.lane, extm, qm[r0], qm[r1], qm[r2], qm[r3], qm[r4], qm[r5], qm[r6], qm[r7], qm[r8], lm);
    float np[VEC], nm[VEC], inc[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float cp = qp[r4][j], cm = qm[r4][j];
        inc[j] = d[j] * lp[j];
        np[j] = inc[j] + ((cp + cp) - p1[j]);
        nm[j] = fmaf(d[j], lm[j], (cm + cm) - m1[j]);
    }
    if (C.own) {
        const int64_t o = (int64_t)z * C.plane + (int64_t)C.y * C.pitch + C.x;
        stv<VEC>(P1 + o, np);
        stv<VEC>(M1 + o, nm);
        if constexpr (GRAD) {
            float g[VEC];
            ldv<VEC>(A0 + o, g);
#pragma unroll
            for (int j = 0; j < VEC; ++j) g[j] = fmaf(qm[r4][j], inc[j], g[j]);
            stv<VEC>(A0 + o, g);
        } else if (img_row) {
            float a[VEC], b[VEC];
            ldv<VEC>(A0 + o, a);
            ldv<VEC>(A1 + o, b);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                a[j] = fmaf(qp[r4][j], qm[r4][j], a[j]);
                b[j] = fmaf(qp[r4][j], qp[r4][j], b[j]);
            }
            stv<VEC>(A0 + o, a);
            stv<VEC>(A1 + o, b);
        }
    }
}

#define RTM_MARCH3(ROWCALL)                                                                    \
    for (int z = T.z0; z < T.z1; z += kZUnroll) {                                              \
        ROWCALL(0, z); ROWCALL(1, z + 1); ROWCALL(2, z + 2); ROWCALL(3, z + 3);                \
        ROWCALL(4, z + 4); ROWCALL(5, z + 5); ROWCALL(6, z + 6); ROWCALL(7, z + 7);            \
        ROWCALL(8, z + 8);                                                                     \
    }

template <int VEC>
__device__ __forceinline__ Ctx3<VEC> make_ctx3(const ShotDev &S, const Tile3D &T)
{
    Ctx3<VEC> C;
    C.pitch = S.L.pitch;
    C.plane = S.L.plane;
    C.NX = S.L.NX;
    C.NY = S.L.NY;
    C.lane = threadIdx.x & 63;
    C.w = threadIdx.x >> 6;
    C.x0 = T.x0;
    C.y0 = T.y0;
    C.x = T.x0 + C.lane * VEC;
    C.y = T.y0 + C.w;
    C.liveX = C.x < C.NX + kRadius;
    C.rowlive = C.y < C.NY + kRadius;
    C.live = C.liveX && C.rowlive;
    C.own = C.x < C.NX && C.y < C.NY;
    return C;
}

// Does this wave-lane own padded cell (y, x) of the tile?
template <int VEC>
__device__ __forceinline__ bool owns3(const Ctx3<VEC> &C, int y, int x)
{
    return y == C.y && x >= C.x && x < C.x + VEC;
}

}  // namespace

// Forward step n (see the 2-D kernel): tiles of 64*VEC x TY x (z1 - z0).
// Workgroups past the stencil slots record d^n = R p^n, one receiver task
// of 64 per wavefront.
template <int VEC, int TY>
__global__ __launch_bounds__(64 * TY) void fwd3d_kernel(const ShotDev *__restrict__ shots,
                                                        const Tile3D *__restrict__ tiles, int ntiles, int nslots,
                                                        const InjEnt *__restrict__ ents,
                                                        const Contrib *__restrict__ cont,
                                                        const SampleTask *__restrict__ stasks, int nsample, int n)
{
    __shared__ Lds<VEC, TY> L;
    const int b = blockIdx.x;
    if (b >= nslots) {
        const int task = (b - nslots) * TY + (int)(threadIdx.x >> 6);
        if (task < nsample) sample_body(shots, stasks[task], n, n & 1, (int)(threadIdx.x & 63));
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;
    const Tile3D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const Ctx3<VEC> C = make_ctx3<VEC>(S, T);
    const gfloat *pc = gp(S.fld[n & 1] + S.L.org);
    gfloat *po = gp(S.fld[(n + 1) & 1] + S.L.org);
    const gfloat *Dp = gp(S.Dp + S.L.org);
    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) plane_prefetch<VEC>(C, pc, T.z0 - 4 + i, q[i]);
    FieldNext<VEC, TY> nx;
    float nold[VEC], nd[VEC];
    field_prefetch<VEC, TY>(C, pc, T.z0, nx);
    plane_prefetch<VEC>(C, po, T.z0, nold);
    plane_prefetch<VEC>(C, Dp, T.z0, nd);
#define RTM_FWD3(SS, ZZ) fwd3_plane<VEC, TY, SS>(C, L, pc, po, Dp, q, nx, nold, nd, ZZ, T.z0, T.z1)
    RTM_MARCH3(RTM_FWD3)
#undef RTM_FWD3
    const float *wav = S.wav + n;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns3<VEC>(C, E.y, E.x)) {
            const int64_t o = (int64_t)E.z * C.plane + (int64_t)E.y * C.pitch + E.x;
            po[o] = fmaf(Dp[o], inj_sum(E, cont, wav), po[o]);
        }
    }
}

// Reverse step k (see the 2-D kernel), with LDS copies of both fields.
template <int VEC, int TY, bool GRAD>
__global__ __launch_bounds__(64 * TY) void rev3d_kernel(const ShotDev *__restrict__ shots,
                                                        const Tile3D *__restrict__ tiles, int ntiles, int nslots,
                                                        const InjEnt *__restrict__ ents,
                                                        const Contrib *__restrict__ cont, int k, int reinject,
                                                        float *__restrict__ wadj)
{
    __shared__ Lds<VEC, TY> LP, LM;
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile3D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const Ctx3<VEC> C = make_ctx3<VEC>(S, T);
    const gfloat *P0 = gp(S.fld[k & 1] + S.L.org);
    gfloat *P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    const gfloat *M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    gfloat *M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    const gfloat *Dp = gp(S.Dp + S.L.org);
    gfloat *A0 = gp(S.acc0 + S.L.org);
    gfloat *A1 = GRAD ? nullptr : gp(S.acc1 + S.L.org);
    const bool img_lane = C.x + VEC > S.ix0 && C.x < S.ix1 && C.y >= S.iy0 && C.y < S.iy1;
    float qp[9][VEC], qm[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        plane_prefetch<VEC>(C, P0, T.z0 - 4 + i, qp[i]);
        plane_prefetch<VEC>(C, M0, T.z0 - 4 + i, qm[i]);
    }
    FieldNext<VEC, TY> npf, nmf;
    float np1[VEC], nm1[VEC], nd[VEC];
    field_prefetch<VEC, TY>(C, P0, T.z0, npf);
    field_prefetch<VEC, TY>(C, M0, T.z0, nmf);
    plane_prefetch<VEC>(C, P1, T.z0, np1);
    plane_prefetch<VEC>(C, M1, T.z0, nm1);
    plane_prefetch<VEC>(C, Dp, T.z0, nd);
#define RTM_REV3(SS, ZZ) \
    rev3_plane<VEC, TY, GRAD, SS>(C, LP, LM, P0, P1, M0, M1, Dp, A0, A1, qp, qm, npf, nmf, np1, nm1, nd, ZZ, T.z0, \
                                  T.z1, img_lane && (ZZ) >= S.iz0 && (ZZ) < S.iz1)
    RTM_MARCH3(RTM_REV3)
#undef RTM_REV3
    const float *wav = S.wav + k;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns3<VEC>(C, E.y, E.x)) {
            const int64_t o = (int64_t)E.z * C.plane + (int64_t)E.y * C.pitch + E.x;
            const float ds = Dp[o] * inj_sum(E, cont, wav);
            if (reinject) P1[o] = P1[o] + ds;
            if (GRAD) A0[o] = fmaf(M0[o], ds, A0[o]);
            if (wadj) {
                float wsum = 0.f;
                for (int c = E.cbeg; c < E.cend; ++c) wsum += cont[c].w;
                wadj[(int64_t)k * kMaxNodes + E.slot] = wsum * M0[o];
            }
        }
    }
    inject_nodes(M1, Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)k * S.nrec, C.plane, C.pitch);
}

// Receiver wavefield alone, for migration with a stored source wavefield
// (see the 2-D kernel): the forward plane update applied to mu, with the
// imaging sums at a stored level taking p^k from the dense snapshot (IMG).
template <int VEC, int TY, bool IMG>
__global__ __launch_bounds__(64 * TY) void recv3d_kernel(const ShotDev *__restrict__ shots,
                                                         const Tile3D *__restrict__ tiles, int ntiles, int nslots,
                                                         const InjEnt *__restrict__ ents,
                                                         const Contrib *__restrict__ cont, int k,
                                                         const float *__restrict__ snap)
{
    __shared__ Lds<VEC, TY> L;
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile3D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const Ctx3<VEC> C = make_ctx3<VEC>(S, T);
    const gfloat *pc = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);  // mu^{k+1}
    gfloat *po = gp(S.fld[2 + (k & 1)] + S.L.org);              // mu^{k+2} -> mu^k
    const gfloat *Dp = gp(S.Dp + S.L.org);
    gfloat *A0 = gp(S.acc0 + S.L.org), *A1 = gp(S.acc1 + S.L.org);
    const bool img = IMG && C.own && C.x + VEC > S.ix0 && C.x < S.ix1 && C.y >= S.iy0 && C.y < S.iy1;
    const SnapImg I{snap, S.ix1 - S.ix0, S.iy1 - S.iy0, S.ix0, S.ix1, S.iy0, S.iz0};
    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) plane_prefetch<VEC>(C, pc, T.z0 - 4 + i, q[i]);
    FieldNext<VEC, TY> nx;
    float nold[VEC], nd[VEC];
    field_prefetch<VEC, TY>(C, pc, T.z0, nx);
    plane_prefetch<VEC>(C, po, T.z0, nold);
    plane_prefetch<VEC>(C, Dp, T.z0, nd);
#define RTM_RECV3(SS, ZZ)                                                                                       \
    fwd3_plane<VEC, TY, SS>(C, L, pc, po, Dp, q, nx, nold, nd, ZZ, T.z0, T.z1);                                  \
    if constexpr (IMG)                                                                                           \
        if (img && (ZZ) >= S.iz0 && (ZZ) < S.iz1)                                                                \
            snap_image<VEC>(I, A0, A1, (int64_t)(ZZ) * C.plane + (int64_t)C.y * C.pitch + C.x, ZZ, C.y, C.x,     \
                            q[((SS) + 4) % 9]);
    RTM_MARCH3(RTM_RECV3)
#undef RTM_RECV3
    inject_nodes(po, Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)k * S.nrec, C.plane, C.pitch);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

hipError_t launch_fwd3d(int vec, int ty, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st)
{
    const int nsb = (nsample + ty - 1) / ty;
    dim3 grid(nslots + nsb), block(64 * ty);
#define RTM_F3(V, Y) \
    hipLaunchKernelGGL((fwd3d_kernel<V, Y>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n)
    if (ty == 4) {
        switch (vec) {
        case 1: RTM_F3(1, 4); break;
        case 2: RTM_F3(2, 4); break;
        case 4: RTM_F3(4, 4); break;
        default: return hipErrorInvalidValue;
        }
    } else if (ty == 8) {
        switch (vec) {
        case 1: RTM_F3(1, 8); break;
        case 2: RTM_F3(2, 8); break;
        case 4: RTM_F3(4, 8); break;
        default: return hipErrorInvalidValue;
        }
    } else if (ty == 16) {
        switch (vec) {
        case 1: RTM_F3(1, 16); break;
        case 2: RTM_F3(2, 16); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef RTM_F3
    return hipGetLastError();
}

hipError_t launch_rev3d(int vec, int ty, bool grad, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st)
{
    dim3 grid(nslots), block(64 * ty);
#define RTM_R3(V, Y, G) \
    hipLaunchKernelGGL((rev3d_kernel<V, Y, G>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject, wadj)
#define RTM_R3V(Y, G)                          \
    switch (vec) {                             \
    case 1: RTM_R3(1, Y, G); break;            \
    case 2: RTM_R3(2, Y, G); break;            \
    case 4: RTM_R3(4, Y, G); break;            \
    default: return hipErrorInvalidValue;      \
    }
    if (ty == 4) {
        if (grad) { RTM_R3V(4, true) } else { RTM_R3V(4, false) }
    } else if (ty == 8) {
        if (grad) { RTM_R3V(8, true) } else { RTM_R3V(8, false) }
    } else if (ty == 16 && vec == 1) {
        if (grad) { RTM_R3(1, 16, true); } else { RTM_R3(1, 16, false); }
    } else {
        return hipErrorInvalidValue;
    }
#undef RTM_R3V
#undef RTM_R3
    return hipGetLastError();
}

hipError_t launch_recv3d(int vec, int ty, const ShotDev *shots, const Tile3D *tiles, int ntiles, int nslots,
                         const InjEnt *ents, const Contrib *cont, int k, const float *snap, hipStream_t st)
{
    dim3 grid(nslots), block(64 * ty);
#define RTM_RC3(V, Y)                                                                                              \
    if (snap)                                                                                                      \
        hipLaunchKernelGGL((recv3d_kernel<V, Y, true>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, \
                           snap);                                                                                  \
    else                                                                                                           \
        hipLaunchKernelGGL((recv3d_kernel<V, Y, false>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, \
                           k, snap)
#define RTM_RC3V(Y)                            \
    switch (vec) {                             \
    case 1: RTM_RC3(1, Y); break;              \
    case 2: RTM_RC3(2, Y); break;              \
    case 4: RTM_RC3(4, Y); break;              \
    default: return hipErrorInvalidValue;      \
    }
    if (ty == 4) {
        RTM_RC3V(4)
    } else if (ty == 8) {
        RTM_RC3V(8)
    } else if (ty == 16) {
        switch (vec) {
        case 1: RTM_RC3(1, 16); break;
        case 2: RTM_RC3(2, 16); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef RTM_RC3V
#undef RTM_RC3
    return hipGetLastError();
}

}  // namespace rtm
