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

// Writes this wave's centre row and its share of the 8 y-halo rows of plane
// z into LDS buffer `buf`.
template <int VEC, int TY>
__device__ __forceinline__ void lds_fill(Lds<VEC, TY> &L, int buf, int w, int lane, const float (&c)[VEC],
                                         const gfloat *plane_z, int64_t pitch, int x, int y0, int NY, bool liveX)
{
#pragma unroll
    for (int j = 0; j < VEC; ++j) L.row[buf][4 + w][lane * VEC + j] = c[j];
#pragma unroll
    for (int h = w; h < 8; h += TY) {
        const int yh = h < 4 ? y0 - 4 + h : y0 + TY + (h - 4);
        const int slot = h < 4 ? h : TY + 4 + (h - 4);
        float v[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) v[j] = 0.f;
        if (liveX && yh < NY + kRadius) ldv<VEC>(plane_z + (int64_t)yh * pitch + x, v);
#pragma unroll
        for (int j = 0; j < VEC; ++j) L.row[buf][slot][lane * VEC + j] = v[j];
    }
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
struct Ctx3 {
    int64_t pitch, plane;
    int x, x0, y, y0, NX, NY, lane, w;
    bool liveX, live, own;
};

template <int VEC, int TY, int S>
__device__ __forceinline__ void fwd3_plane(const Ctx3<VEC> &C, Lds<VEC, TY> &L, const gfloat *pc, gfloat *po,
                                           const gfloat *Dp, float (&q)[9][VEC], int z, int z0)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int buf = (z - z0) & 1;
    const int64_t o = (int64_t)z * C.plane + (int64_t)C.y * C.pitch + C.x;
    float old[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q[r8][j] = old[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(pc + o + 4 * C.plane, q[r8]);
        ldv<VEC>(po + o, old);
        ldv<VEC>(Dp + o, d);
    }
    lds_fill<VEC, TY>(L, buf, C.w, C.lane, q[r4], pc + (int64_t)z * C.plane, C.pitch, C.x, C.y0, C.NY, C.liveX);
    float hl[4], hr[4], ext[VEC + 8];
    load_halo<VEC>(pc + (int64_t)z * C.plane + (int64_t)C.y * C.pitch, C.x0, C.NX, C.lane, hl, hr,
                   C.y < C.NY + kRadius);
    exchange_row<VEC>(q[r4], hl, hr, ext);
    __syncthreads();
    float lap[VEC], out[VEC];
    lap3<VEC, TY>(L, buf, C.w, C.lane, ext, q[r0], q[r1], q[r2], q[r3], q[r4], q[r5], q[r6], q[r7], q[r8], lap);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q[r4][j];
        out[j] = fmaf(d[j], lap[j], (c + c) - old[j]);
    }
    if (C.own) stv<VEC>(po + o, out);
}

template <int VEC, int TY, bool GRAD, int S>
__device__ __forceinline__ void rev3_plane(const Ctx3<VEC> &C, Lds<VEC, TY> &LP, Lds<VEC, TY> &LM,
                                           const gfloat *P0, gfloat *P1, const gfloat *M0, gfloat *M1,
                                           const gfloat *Dp, gfloat *A0, gfloat *A1, float (&qp)[9][VEC],
                                           float (&qm)[9][VEC], int z, int z0, bool img_row)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int buf = (z - z0) & 1;
    const int64_t o = (int64_t)z * C.plane + (int64_t)C.y * C.pitch + C.x;
    const int64_t ro = (int64_t)z * C.plane + (int64_t)C.y * C.pitch;
    float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) qp[r8][j] = qm[r8][j] = p1[j] = m1[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(P0 + o + 4 * C.plane, qp[r8]);
        ldv<VEC>(M0 + o + 4 * C.plane, qm[r8]);
        ldv<VEC>(P1 + o, p1);
        ldv<VEC>(M1 + o, m1);
        ldv<VEC>(Dp + o, d);
    }
    lds_fill<VEC, TY>(LP, buf, C.w, C.lane, qp[r4], P0 + (int64_t)z * C.plane, C.pitch, C.x, C.y0, C.NY, C.liveX);
    lds_fill<VEC, TY>(LM, buf, C.w, C.lane, qm[r4], M0 + (int64_t)z * C.plane, C.pitch, C.x, C.y0, C.NY, C.liveX);
    const bool rowlive = C.y < C.NY + kRadius;
    float hl[4], hr[4], extp[VEC + 8], extm[VEC + 8];
    load_halo<VEC>(P0 + ro, C.x0, C.NX, C.lane, hl, hr, rowlive);
    exchange_row<VEC>(qp[r4], hl, hr, extp);
    load_halo<VEC>(M0 + ro, C.x0, C.NX, C.lane, hl, hr, rowlive);
    exchange_row<VEC>(qm[r4], hl, hr, extm);
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
    C.live = C.liveX && C.y < C.NY + kRadius;
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
        if (task < nsample) sample_body(shots, stasks[task], n, (int)(threadIdx.x & 63));
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
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[i][j] = 0.f;
        if (C.live) ldv<VEC>(pc + (int64_t)(T.z0 - 4 + i) * C.plane + (int64_t)C.y * C.pitch + C.x, q[i]);
    }
#define RTM_FWD3(SS, ZZ) fwd3_plane<VEC, TY, SS>(C, L, pc, po, Dp, q, ZZ, T.z0)
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
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[i][j] = qm[i][j] = 0.f;
        if (C.live) {
            const int64_t o = (int64_t)(T.z0 - 4 + i) * C.plane + (int64_t)C.y * C.pitch + C.x;
            ldv<VEC>(P0 + o, qp[i]);
            ldv<VEC>(M0 + o, qm[i]);
        }
    }
#define RTM_REV3(SS, ZZ) \
    rev3_plane<VEC, TY, GRAD, SS>(C, LP, LM, P0, P1, M0, M1, Dp, A0, A1, qp, qm, ZZ, T.z0, \
                                  img_lane && (ZZ) >= S.iz0 && (ZZ) < S.iz1)
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
    const float *sig = S.sig + (int64_t)k * S.nrec;
    for (int e = T.rbeg; e < T.rend; ++e) {
        const InjEnt E = ents[e];
        if (owns3<VEC>(C, E.y, E.x)) {
            const int64_t o = (int64_t)E.z * C.plane + (int64_t)E.y * C.pitch + E.x;
            M1[o] = fmaf(Dp[o], inj_sum(E, cont, sig), M1[o]);
        }
    }
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
    } else {
        return hipErrorInvalidValue;
    }
#undef RTM_R3V
#undef RTM_R3
    return hipGetLastError();
}

}  // namespace rtm
