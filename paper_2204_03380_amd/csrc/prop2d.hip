// 2-D propagation kernels for gfx950.
//
// One wavefront (64 lanes) owns a strip of 64 * VEC consecutive x cells and
// marches down the rows [z0, z1) of its tile.  Each lane keeps the nine rows
// z-4 .. z+4 of its VEC cells in registers (a register queue), so every
// stored value of the input field is read from memory once per tile plus the
// 8-row overlap with the tiles above and below.  The march is unrolled by
// nine so that the queue rotates by register renaming, not by moves.  The
// x-neighbours of the centre row come from the adjacent lanes through DPP
// wave shifts; lanes 0 and 63 supply the 4-cell halo at the strip ends with
// one extra load.
//
// The stencil is evaluated as
//   L p_i = sum_axis sum_{m=1..4} c_m ((p_{i+m} + p_{i-m}) - 2 p_i),
// algebraically the 8th-order Laplacian of Sec. 3, but exactly zero on a
// constant field in FP32: the rounded weights then cannot add a spurious
// mass term, which would otherwise accumulate into a phase error of ~1e-3
// after a few thousand steps.
//
// Fields are stored with a zero halo and the scaled velocity term
// D' = (v dt / h)^2 is zero there, so updating a halo cell reproduces zero;
// lanes past the grid edge only have to skip their loads and stores.
#include <atomic>

#include "stencil.h"

namespace rtm {
namespace {

// --------------------------------------------------------------------------
// Forward step
// --------------------------------------------------------------------------

template <int VEC>
struct FwdCtx {
    const gfloat *pc;  // p^n
    gfloat *po;        // p^{n-1}, overwritten by p^{n+1}
    const gfloat *Dp;
    int64_t pitch;
    int x, x0, NX, lane, w;  // x0: first cell of this wave's strip; w: wave in the workgroup
    bool live, own;
};

// Row z of the march.  Queue slot (S + i) % 9 holds row z - 4 + i; the slot
// of row z + 4 is refilled here.  With TX strips per workgroup the inner
// strip ends come from the edge ring (slot S holds row z); the workgroup
// meets at a barrier every third row, which orders each ring write (row
// z + 4, end of this step) before its read four steps later and each read
// before the slot is rewritten five steps later.
// The one-step forward row (forward and receiver-only kernels) with one
// strip per workgroup fetches each row's strip-end halo one march step early
// (hc: the halo of row z, fetched at row z - 1), as the two-step kernels do:
// 326 -> 339 us without it for 48 shots at vec 1.  The one-step reverse
// kernel keeps the in-step load (no consistent gain: 854 -> 874 us at vec 1,
// 868 -> 849 at vec 4).
template <int VEC, int TX>
constexpr bool ahead1() { return TX == 1 && VEC != 2; }

// Strip-end halo of row z into hl / hr: the early-fetched one (then fetch
// row z + 1's, always a stored row as z < NZr) or a load now.
template <int VEC, int TX, bool AHEAD>
__device__ __forceinline__ void row_halo(const gfloat *f, int64_t pitch, int z, int x0, int NX, int lane, int w,
                                         f4v &hc, float (&hl)[4], float (&hr)[4])
{
    if constexpr (AHEAD) {
        const f4v t = hc;
        hc = halo_fetch<VEC>(f + (int64_t)(z + 1) * pitch, x0, NX, lane, true);
        halo_split(t, lane, hl, hr);
    } else {
        load_halo_outer<VEC>(f + (int64_t)z * pitch, x0, NX, lane, w == 0, w == TX - 1, hl, hr);
    }
}

template <int VEC, int TX, int S>
__device__ __forceinline__ void fwd_row(const FwdCtx<VEC> &C, float (&q)[9][VEC], int z, EdgeRing<TX> &R, f4v &hc)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    if constexpr (TX > 1 && S % 3 == 0) __syncthreads();
    const int64_t o = (int64_t)z * C.pitch + C.x;
    float old[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q[r8][j] = old[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(C.pc + o + 4 * C.pitch, q[r8]);
        ldv<VEC>(C.po + o, old);
        ldv<VEC>(C.Dp + o, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    row_halo<VEC, TX, ahead1<VEC, TX>()>(C.pc, C.pitch, z, C.x0, C.NX, C.lane, C.w, hc, hl, hr);
    ring_get<TX>(R, S, C.w, C.lane, hl, hr);
    exchange_row<VEC>(q[r4], hl, hr, ext);
    float out[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, q[r3][j], q[r5][j], q[r2][j], q[r6][j], q[r1][j], q[r7][j], q[r0][j], q[r8][j]);
        out[j] = fmaf(d[j], lap, c2 - old[j]);
    }
    if (C.own) stv<VEC>(C.po + o, out);
    if constexpr (TX > 1) ring_put<VEC, TX>(R, (S + 4) % 9, C.w, C.lane, q[r8]);
}

// --------------------------------------------------------------------------
// Reverse step
// --------------------------------------------------------------------------

template <int VEC>
struct RevCtx {
    const gfloat *P0;  // p^k
    gfloat *P1;        // p^{k+1} -> p^{k-1}
    const gfloat *M0;  // mu^{k+1}
    gfloat *M1;        // mu^{k+2} -> mu^k
    const gfloat *Dp;
    gfloat *A0, *A1;   // num, den | G
    int64_t pitch;
    int x, x0, NX, lane, w, iz0, iz1;
    bool live, own, own_img, reinject;
};

template <int VEC, bool GRAD, int TX, int S>
__device__ __forceinline__ void rev_row(const RevCtx<VEC> &C, float (&qp)[9][VEC], float (&qm)[9][VEC], int z,
                                        EdgeRing<TX> &RP, EdgeRing<TX> &RM, f4v &hp, f4v &hm)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    if constexpr (TX > 1 && S % 3 == 0) __syncthreads();
    const int64_t o = (int64_t)z * C.pitch + C.x;
    float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) qp[r8][j] = qm[r8][j] = p1[j] = m1[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(C.P0 + o + 4 * C.pitch, qp[r8]);
        ldv<VEC>(C.M0 + o + 4 * C.pitch, qm[r8]);
        ldv_s<VEC>(C.P1 + o, p1);
        ldv_s<VEC>(C.M1 + o, m1);
        ldv_s<VEC>(C.Dp + o, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    float np[VEC], nm[VEC], inc[VEC];
    row_halo<VEC, TX, false>(C.P0, C.pitch, z, C.x0, C.NX, C.lane, C.w, hp, hl, hr);
    ring_get<TX>(RP, S, C.w, C.lane, hl, hr);
    exchange_row<VEC>(qp[r4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = qp[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, qp[r3][j], qp[r5][j], qp[r2][j], qp[r6][j], qp[r1][j], qp[r7][j], qp[r0][j], qp[r8][j]);
        inc[j] = d[j] * lap;                 // gradient term (GRAD)
        np[j] = fmaf(d[j], lap, c2 - p1[j]);  // same rounding as the two-step kernel
    }
    if (C.own) stv<VEC>(C.P1 + o, np);
    row_halo<VEC, TX, false>(C.M0, C.pitch, z, C.x0, C.NX, C.lane, C.w, hm, hl, hr);
    ring_get<TX>(RM, S, C.w, C.lane, hl, hr);
    exchange_row<VEC>(qm[r4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = qm[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, qm[r3][j], qm[r5][j], qm[r2][j], qm[r6][j], qm[r1][j], qm[r7][j], qm[r0][j], qm[r8][j]);
        nm[j] = fmaf(d[j], lap, c2 - m1[j]);
    }
    if (C.own) stv<VEC>(C.M1 + o, nm);
    if constexpr (GRAD) {
        if (C.own) {
            float g[VEC];
            ldv<VEC>(C.A0 + o, g);
#pragma unroll
            for (int j = 0; j < VEC; ++j) g[j] = fmaf(qm[r4][j], inc[j], g[j]);
            stv<VEC>(C.A0 + o, g);
        }
    } else {
        if (z >= C.iz0 && z < C.iz1 && C.own_img) {
            float a[VEC], b[VEC];
            ldv_s<VEC>(C.A0 + o, a);
            ldv_s<VEC>(C.A1 + o, b);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                a[j] = fmaf(qp[r4][j], qm[r4][j], a[j]);
                b[j] = fmaf(qp[r4][j], qp[r4][j], b[j]);
            }
            stv_s<VEC>(C.A0 + o, a);
            stv_s<VEC>(C.A1 + o, b);
        }
    }
    if constexpr (TX > 1) {
        ring_put<VEC, TX>(RP, (S + 4) % 9, C.w, C.lane, qp[r8]);
        ring_put<VEC, TX>(RM, (S + 4) % 9, C.w, C.lane, qm[r8]);
    }
}

// Runs ROWCALL(S, z) over the tile's rows, nine per trip (z1 - z0 is a
// multiple of nine), so that S = (z - z0) mod 9 is a compile-time constant.
#define RTM_MARCH(ROWCALL)                                                                     \
    for (int z = T.z0; z < T.z1; z += kZUnroll) {                                              \
        ROWCALL(0, z); ROWCALL(1, z + 1); ROWCALL(2, z + 2); ROWCALL(3, z + 3);                \
        ROWCALL(4, z + 4); ROWCALL(5, z + 5); ROWCALL(6, z + 6); ROWCALL(7, z + 7);            \
        ROWCALL(8, z + 8);                                                                     \
    }

}  // namespace

// Forward step n of every tile:  p^{n+1} = 2 p^n - p^{n-1} + D' (L p^n + s^n),
// written over p^{n-1}; workgroups past the stencil slots record d^n = R p^n.
// The source term is added to the stored value after the march by the lane
// that stored it (same thread, so program order makes the value visible).
// A workgroup of TX wavefronts covers TX adjacent strips of one tile.
template <int VEC, int TX>
__device__ __forceinline__ void fwd2d_tile(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles, int t,
                                           const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int n,
                                           int w, int lane, EdgeRing<TX> &ring)
{
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    FwdCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.pc = gp(S.fld[n & 1] + S.L.org);
    C.po = gp(S.fld[(n + 1) & 1] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.lane = lane;
    C.w = w;
    C.x0 = T.x0 + w * 64 * VEC;
    C.x = C.x0 + lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;

    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[i][j] = 0.f;
        if (C.live) ldv<VEC>(C.pc + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, q[i]);
        // rows z0 .. z0 + 3 (queue slots 4..7, ring slots 0..3); the first
        // march step opens with a barrier
        if constexpr (TX > 1)
            if (i >= 4) ring_put<VEC, TX>(ring, i - 4, w, lane, q[i]);
    }
    f4v hc = halo_fetch<VEC>(C.pc + (int64_t)T.z0 * C.pitch, C.x0, C.NX, lane, ahead1<VEC, TX>());
#define RTM_FWD_ROW(SS, ZZ) fwd_row<VEC, TX, SS>(C, q, ZZ, ring, hc)
    RTM_MARCH(RTM_FWD_ROW)
#undef RTM_FWD_ROW
    // Source injection: p^{n+1} += D' s^n at the source nodes of this tile.
    const float *wav = S.wav + n;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, C.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            C.po[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav), C.po[o]);
        }
    }
}

template <int VEC, int TX>
__global__ __launch_bounds__(64 * TX) void fwd2d_kernel(const ShotDev *__restrict__ shots,
                                                        const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                        const InjEnt *__restrict__ ents,
                                                        const Contrib *__restrict__ cont,
                                                        const SampleTask *__restrict__ stasks, int nsample, int n)
{
    const int b = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (b >= nslots) {
        const int task = (b - nslots) * TX + w;
        if (task < nsample) sample_body(shots, stasks[task], n, n & 1, lane);
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;  // whole workgroup
    __shared__ EdgeRing<TX> ring;
    fwd2d_tile<VEC, TX>(shots, tiles, t, ents, cont, n, w, lane, ring);
}

// Reverse step k of every tile, Eqs. (2), (3) and (6) in one pass:
//   p^{k-1} = 2 p^k - p^{k+1} + D' (L p^k + s^k)         (reconstruction)
//   mu^k    = 2 mu^{k+1} - mu^{k+2} + D' (L mu^{k+1} + r^k)  (receiver field)
// and either the imaging sums num += p^k mu^{k+1}, den += (p^k)^2 on the
// interior (GRAD = false) or the gradient sum G += mu^{k+1} D' (L p^k + s^k)
// on the whole padded grid (GRAD = true).  With reinject = 0 the source term
// is left out of the reconstruction (Eq. (6) as written).  The source and
// receiver terms are added after the march by the lanes that stored the
// cells.  When wadj is non-null, those lanes also write each source node's
// coefficient times mu^{k+1} to wadj[k * kMaxNodes + node].
// With one float per lane the reverse kernel fits in 64 registers; asking
// for 8 waves per SIMD then hides more latency (measured: 4.5 vs 4.2 TB/s
// on 16 shots of the 2301 x 751 grid).  Wider lanes would spill.
// rev2d_kernel's tile body as a function, for the persistent pass.  The
// kernel keeps its own copy of the body: compiled through this function,
// its one-float-per-lane instance (held to 64 registers for 8 waves per
// SIMD) spills 156 bytes per lane, while the copy fits.
template <int VEC, bool GRAD, int TX>
__device__ __forceinline__ void rev2d_tile(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles, int t,
                                           const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int k,
                                           int reinject, float *__restrict__ wadj, int w, int lane,
                                           EdgeRing<TX> &ring_p, EdgeRing<TX> &ring_m)
{
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    RevCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.P0 = gp(S.fld[k & 1] + S.L.org);
    C.P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    C.M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    C.M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.A0 = gp(S.acc0 + S.L.org);
    C.A1 = GRAD ? nullptr : gp(S.acc1 + S.L.org);
    C.lane = lane;
    C.w = w;
    C.x0 = T.x0 + w * 64 * VEC;
    C.x = C.x0 + lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;
    // Lanes whose cells overlap the interior accumulate the image sums (their
    // other cells lie in the band or halo, whose sums are never read).
    C.own_img = C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    C.iz0 = S.iz0;
    C.iz1 = S.iz1;
    C.reinject = reinject != 0;

    float qp[9][VEC], qm[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[i][j] = qm[i][j] = 0.f;
        if (C.live) {
            ldv<VEC>(C.P0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qp[i]);
            ldv<VEC>(C.M0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qm[i]);
        }
        if constexpr (TX > 1)
            if (i >= 4) {
                ring_put<VEC, TX>(ring_p, i - 4, w, lane, qp[i]);
                ring_put<VEC, TX>(ring_m, i - 4, w, lane, qm[i]);
            }
    }
    f4v hp = f4v{0.f, 0.f, 0.f, 0.f}, hm = hp;  // (the reverse rows load their halo in-step)
#define RTM_REV_ROW(SS, ZZ) rev_row<VEC, GRAD, TX, SS>(C, qp, qm, ZZ, ring_p, ring_m, hp, hm)
    RTM_MARCH(RTM_REV_ROW)
#undef RTM_REV_ROW
    // Source term at step k: reconstruction (re-injection), gradient, wavelet adjoint.
    const float *wav = S.wav + k;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, C.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            const float sv = inj_sum(E, cont, wav);
            if (C.reinject) C.P1[o] = fmaf(C.Dp[o], sv, C.P1[o]);
            if (GRAD) C.A0[o] = fmaf(C.M0[o], C.Dp[o] * sv, C.A0[o]);
            if (wadj) {
                float wsum = 0.f;
                for (int c = E.cbeg; c < E.cend; ++c) wsum += cont[c].w;
                wadj[(int64_t)k * kMaxNodes + E.slot] = wsum * C.M0[o];
            }
        }
    }
    // Receiver term: mu^k += D' R^T g^k.
    inject_nodes(C.M1, C.Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)k * S.nrec, C.pitch, C.pitch);
}

template <int VEC, bool GRAD, int TX>
__global__ __launch_bounds__(64 * TX) __attribute__((amdgpu_waves_per_eu(VEC == 1 ? 8 : 1, 8)))
void rev2d_kernel(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                  const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int k, int reinject,
                  float *__restrict__ wadj)
{
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;  // whole workgroup
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ EdgeRing<TX> ring_p, ring_m;
    RevCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.P0 = gp(S.fld[k & 1] + S.L.org);
    C.P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    C.M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    C.M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.A0 = gp(S.acc0 + S.L.org);
    C.A1 = GRAD ? nullptr : gp(S.acc1 + S.L.org);
    C.lane = lane;
    C.w = w;
    C.x0 = T.x0 + w * 64 * VEC;
    C.x = C.x0 + lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;
    // Lanes whose cells overlap the interior accumulate the image sums (their
    // other cells lie in the band or halo, whose sums are never read).
    C.own_img = C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    C.iz0 = S.iz0;
    C.iz1 = S.iz1;
    C.reinject = reinject != 0;

    float qp[9][VEC], qm[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[i][j] = qm[i][j] = 0.f;
        if (C.live) {
            ldv<VEC>(C.P0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qp[i]);
            ldv<VEC>(C.M0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qm[i]);
        }
        if constexpr (TX > 1)
            if (i >= 4) {
                ring_put<VEC, TX>(ring_p, i - 4, w, lane, qp[i]);
                ring_put<VEC, TX>(ring_m, i - 4, w, lane, qm[i]);
            }
    }
    f4v hp = f4v{0.f, 0.f, 0.f, 0.f}, hm = hp;  // (the reverse rows load their halo in-step)
#define RTM_REV_ROW(SS, ZZ) rev_row<VEC, GRAD, TX, SS>(C, qp, qm, ZZ, ring_p, ring_m, hp, hm)
    RTM_MARCH(RTM_REV_ROW)
#undef RTM_REV_ROW
    // Source term at step k: reconstruction (re-injection), gradient, wavelet adjoint.
    const float *wav = S.wav + k;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, C.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            const float sv = inj_sum(E, cont, wav);
            if (C.reinject) C.P1[o] = fmaf(C.Dp[o], sv, C.P1[o]);
            if (GRAD) C.A0[o] = fmaf(C.M0[o], C.Dp[o] * sv, C.A0[o]);
            if (wadj) {
                float wsum = 0.f;
                for (int c = E.cbeg; c < E.cend; ++c) wsum += cont[c].w;
                wadj[(int64_t)k * kMaxNodes + E.slot] = wsum * C.M0[o];
            }
        }
    }
    // Receiver term: mu^k += D' R^T g^k.
    inject_nodes(C.M1, C.Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)k * S.nrec, C.pitch, C.pitch);
}

// Receiver wavefield alone, for migration with a stored source wavefield
// (Algorithm 2): mu^k = 2 mu^{k+1} - mu^{k+2} + D' (L mu^{k+1} + r^k), the
// forward row update applied to mu (same operations as the mu half of the
// fused reverse kernel), with the receiver term added after the march.  At
// a stored level (snap non-null: the dense interior p^k) the imaging sums
// num += p^k mu^{k+1}, den += (p^k)^2 take mu^{k+1} from the register queue.
// IMG selects the imaging variant at compile time, so that the other steps
// run the plain forward code.
template <int VEC, int TX, bool IMG>
__global__ __launch_bounds__(64 * TX) void recv2d_kernel(const ShotDev *__restrict__ shots,
                                                         const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                         const InjEnt *__restrict__ ents,
                                                         const Contrib *__restrict__ cont, int k,
                                                         const float *__restrict__ snap)
{
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;  // whole workgroup
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ EdgeRing<TX> ring;
    FwdCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.pc = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);  // mu^{k+1}
    C.po = gp(S.fld[2 + (k & 1)] + S.L.org);        // mu^{k+2} -> mu^k
    C.Dp = gp(S.Dp + S.L.org);
    C.lane = lane;
    C.w = w;
    C.x0 = T.x0 + w * 64 * VEC;
    C.x = C.x0 + lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;
    const bool img = IMG && C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    const SnapImg I{snap, S.ix1 - S.ix0, 1, S.ix0, S.ix1, 0, S.iz0};
    gfloat *A0 = gp(S.acc0 + S.L.org), *A1 = gp(S.acc1 + S.L.org);

    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[i][j] = 0.f;
        if (C.live) ldv<VEC>(C.pc + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, q[i]);
        if constexpr (TX > 1)
            if (i >= 4) ring_put<VEC, TX>(ring, i - 4, w, lane, q[i]);
    }
    f4v hc = halo_fetch<VEC>(C.pc + (int64_t)T.z0 * C.pitch, C.x0, C.NX, lane, ahead1<VEC, TX>());
#define RTM_RECV_ROW(SS, ZZ)                                                                        \
    fwd_row<VEC, TX, SS>(C, q, ZZ, ring, hc);                                                      \
    if constexpr (IMG)                                                                             \
        if (img && (ZZ) >= S.iz0 && (ZZ) < S.iz1)                                                  \
            snap_image<VEC>(I, A0, A1, (int64_t)(ZZ) * C.pitch + C.x, ZZ, 0, C.x, q[((SS) + 4) % 9]);
    RTM_MARCH(RTM_RECV_ROW)
#undef RTM_RECV_ROW
    // Receiver term: mu^k += D' R^T g^k.
    inject_nodes(C.po, C.Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)k * S.nrec, C.pitch, C.pitch);
}

// ---------------------------------------------------------------------------
// Two time steps per launch
// ---------------------------------------------------------------------------
// A wavefront covers the strip [xs, xs + 64 VEC) and owns its inner columns
// [xs + 4, xs + 64 VEC - 4); neighbouring strips overlap by 8 columns.  It
// marches s = 0 .. zseg + 8; at step s it
//  (1) advances the first level at row r1 = z0 - 4 + s on the whole strip,
//      from a register queue q1 of the level read from memory (rows r1 - 4
//      .. r1 + 4) and that level's strip-end halo, as the one-step kernel;
//  (2) advances the second level at row r2 = r1 - 4 from a queue q2 of the
//      first-step rows just computed.  q2 has no halo beyond the strip, so
//      its outer 4 columns are wrong and only owned columns are stored.
// Row r of either level sits in queue slot (r - z0 + 8) mod 9, so both
// queues rotate together.  Injection into the first step happens inside
// the march in every tile whose strip and rows [z0 - 4, z1 + 4) contain the
// node; injection into the second step after the march, by the owner.  The
// arithmetic of every cell equals the one-step kernel's operation for
// operation, so one launch of this kernel gives the same bits as two
// launches of that one, with the level pairs read once and written once per
// two steps (and the levels stay in two sets: read set, write set).
template <int VEC>
__device__ __forceinline__ bool own2(int x, int xs, int NX)
{
    return x >= xs + 4 && x + VEC <= xs + 64 * VEC - 4 && x < NX;
}

// Forward pair: level n+1 from (n, n-1), level n+2 from (n+1, n).
template <int VEC>
struct Fwd2Ctx {
    const gfloat *pc, *pm;  // p^n, p^{n-1} (read set)
    gfloat *w1, *w2;        // p^{n+1}, p^{n+2} (write set)
    const gfloat *Dp;
    const float *wav;       // wavelet from time n
    const InjEnt *ents;
    const Contrib *cont;
    int64_t pitch;
    int x, xs, NX, NZr, lane, z0, z1, e1end;
    bool live, own;
};

// The forward pair fetches each row's strip-end halo one march step early
// at every width (1574 x 534 single shot, vec 1: 9.3 -> 7.0 us per step;
// 48 shots at vec 4: 428 -> 426 us per launch).
template <int VEC, int S>
__device__ __forceinline__ void fwd2_row(const Fwd2Ctx<VEC> &C, float (&q1)[9][VEC], float (&q2)[9][VEC],
                                         float (&qd)[9][VEC], f4v &hc, int s, int &e)
{
    constexpr int a0 = S % 9, a1 = (S + 1) % 9, a2 = (S + 2) % 9, a3 = (S + 3) % 9, a4 = (S + 4) % 9,
                  a5 = (S + 5) % 9, a6 = (S + 6) % 9, a7 = (S + 7) % 9, a8 = (S + 8) % 9;
    const int r1 = C.z0 - 4 + s, r2 = r1 - 4;
    const bool in1 = r1 < C.NZr + kRadius, in_next = r1 + 4 < C.NZr + kRadius;  // stored rows: [-4, NZr + 4)
    const int64_t o1 = (int64_t)r1 * C.pitch + C.x;
    float old[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q1[a8][j] = old[j] = d[j] = 0.f;
    if (C.live && in_next) ldv<VEC>(C.pc + o1 + 4 * C.pitch, q1[a8]);
    if (C.live && in1) {
        ldv<VEC>(C.pm + o1, old);
        ldv<VEC>(C.Dp + o1, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    {
        const f4v t = hc;
        hc = halo_fetch<VEC>(C.pc + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, r1 + 1 < C.NZr + kRadius);
        halo_split(t, C.lane, hl, hr);
    }
    exchange_row<VEC>(q1[a4], hl, hr, ext);
    float v1[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1[a4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, q1[a3][j], q1[a5][j], q1[a2][j], q1[a6][j], q1[a1][j], q1[a7][j], q1[a0][j], q1[a8][j]);
        v1[j] = fmaf(d[j], lap, c2 - old[j]);
    }
    for (; e < C.e1end && C.ents[e].z == r1; ++e) {  // source at time n, row r1
        const InjEnt E = C.ents[e];
        const float sv = inj_sum(E, C.cont, C.wav);
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            if (E.x == C.x + j) v1[j] = fmaf(d[j], sv, v1[j]);
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        q2[a4][j] = v1[j];
        qd[a4][j] = d[j];
    }
    if (C.own && r1 >= C.z0 && r1 < C.z1) stv<VEC>(C.w1 + o1, v1);
    if (s >= 8 && r2 < C.z1) {
        const float hz[4] = {0.f, 0.f, 0.f, 0.f};
        exchange_row<VEC>(q2[a0], hz, hz, ext);
        float v2[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2[a0][j], c2 = c + c;
            float lap =
                d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
            lap += d2(c2, q2[a8][j], q2[a1][j], q2[a7][j], q2[a2][j], q2[a6][j], q2[a3][j], q2[a5][j], q2[a4][j]);
            v2[j] = fmaf(qd[a0][j], lap, c2 - q1[a0][j]);
        }
        if (C.own) stv<VEC>(C.w2 + (int64_t)r2 * C.pitch + C.x, v2);
    }
}

// Runs ROWCALL(S, s) for s = 0 .. nstep - 1 (nstep a multiple of nine).
#define RTM_MARCH2(ROWCALL, NSTEP)                                                             \
    for (int s = 0; s < (NSTEP); s += kZUnroll) {                                              \
        ROWCALL(0, s); ROWCALL(1, s + 1); ROWCALL(2, s + 2); ROWCALL(3, s + 3);                \
        ROWCALL(4, s + 4); ROWCALL(5, s + 5); ROWCALL(6, s + 6); ROWCALL(7, s + 7);            \
        ROWCALL(8, s + 8);                                                                     \
    }

// Steps n and n + 1 of every tile; workgroups past the stencil slots record
// d^{n-1} (n > 0) and d^n from the read set.
template <int VEC>
__global__ __launch_bounds__(64) void fwd2d_t2_kernel(const ShotDev *__restrict__ shots,
                                                      const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                      const InjEnt *__restrict__ ents,
                                                      const Contrib *__restrict__ cont,
                                                      const SampleTask *__restrict__ stasks, int nsample, int n)
{
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    if (b >= nslots) {
        const int t = b - nslots;
        const int level = t < nsample ? n - 1 : n;
        if (level >= 0) sample_body(shots, stasks[t < nsample ? t : t - nsample], level, level & 1, lane);
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    Fwd2Ctx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.NZr = S.L.NZr;
    C.pc = gp(S.fld[n & 1] + S.L.org);
    C.pm = gp(S.fld[(n + 1) & 1] + S.L.org);
    C.w1 = gp(S.fld[4 + ((n + 1) & 1)] + S.L.org);
    C.w2 = gp(S.fld[4 + (n & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.wav = S.wav + n;
    C.ents = ents;
    C.cont = cont;
    C.lane = lane;
    C.xs = T.x0;
    C.x = T.x0 + lane * VEC;
    C.z0 = T.z0;
    C.z1 = T.z1;
    C.e1end = T.s1end;
    C.live = C.x >= -kRadius && C.x < C.NX + kRadius;
    C.own = own2<VEC>(C.x, C.xs, C.NX);

    float q1[9][VEC], q2[9][VEC], qd[9][VEC];
    // level n rows z0 - 8 .. z0 - 1 (rows above -4 do not exist: zero)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q1[i][j] = q2[i][j] = qd[i][j] = 0.f;
        const int r = T.z0 - 8 + i;
        if (C.live && r >= -kRadius) ldv<VEC>(C.pc + (int64_t)r * C.pitch + C.x, q1[i]);
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) q2[8][j] = qd[8][j] = 0.f;
    int e = T.s1beg;
    const int nstep = T.z1 - T.z0 + kZUnroll;
    // strip-end halo of the first march row (z0 - 4 >= -4: stored)
    f4v hc = halo_fetch<VEC>(C.pc + (int64_t)(T.z0 - 4) * C.pitch, C.xs, C.NX, lane, true);
#define RTM_FWD2_ROW(SS, ZZ) fwd2_row<VEC, SS>(C, q1, q2, qd, hc, ZZ, e)
    RTM_MARCH2(RTM_FWD2_ROW, nstep)
#undef RTM_FWD2_ROW
    // Source at time n + 1 into the owned cells of level n + 2.
    const float *wav1 = S.wav + n + 1;
    for (int k = T.sbeg; k < T.send; ++k) {
        const InjEnt E = ents[k];
        if (owns<VEC>(E.x, C.xs, lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            C.w2[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav1), C.w2[o]);
        }
    }
}

// Reverse pair (imaging): steps k and k - 1 of the reconstruction and the
// receiver field, and both steps' imaging sums.
//
// Strip-end halo one row ahead (halo_ahead<VEC>): with four floats per lane
// the kernel runs at one wavefront per SIMD (256 registers), so nothing
// hides the latency of the halo load that each row's stencil waits for;
// fetching it one march step early took the 48-shot reverse pair from 1349
// to 1167 us.  With one float per lane (the narrow tiles of a single small
// shot, whose march is latency-bound) it saves 13% (1574 x 534: 12.2 ->
// 10.7 us per step).  With two floats per lane (three wavefronts per SIMD)
// the eight extra registers cost more than the early fetch gains (1223 ->
// 1264 us), so that shape keeps the in-step load.
template <int VEC>
constexpr bool halo_ahead() { return VEC != 2; }
template <int VEC>
struct Rev2Ctx {
    const gfloat *P0, *P1, *M0, *M1;  // p^k, p^{k+1}, mu^{k+1}, mu^{k+2} (read set)
    gfloat *WP1, *WP2, *WM1, *WM2;    // p^{k-1}, p^{k-2}, mu^k, mu^{k-1} (write set)
    const gfloat *Dp;
    gfloat *A0, *A1;                  // num, den (imaging) or G (gradient)
    const float *wav, *sig;           // wavelet and receiver signal at time k
    const InjEnt *ents;
    const Contrib *cont;
    float *isv;                       // LDS: receiver sums of one row (row_inject)
    int *ihas;
    float *wadj;                      // gradient: wavelet-adjoint samples (nullable)
    int k;
    int64_t pitch;
    int nrec;
    int x, xs, NX, NZr, lane, z0, z1, iz0, iz1, s1end, r1end, send;
    bool live, own, own_img, reinject;
};

// Gradient pair (GRAD): the imaging sums give way to the gradient sum of the
// one-step kernel, G += mu^{k+1} D' (L p^k) on every owned cell, then, on a
// source node, G += mu^{k+1} (D' s^k) and the wavelet-adjoint sample of
// step k, and the same for step k - 1 with mu^k.  Both steps' terms land on
// step two's row r2, where mu^{k+1} and mu^k are step two's previous and
// centre levels; step one's D' L p^k waits four rows in the qa queue.  The
// source nodes are the tile's own list (rows in [z0, z1)), walked in row
// order.  The products and their order are the one-step kernel's.
template <int VEC, bool GRAD, int S>
__device__ __forceinline__ void rev2_row(const Rev2Ctx<VEC> &C, float (&q1p)[9][VEC], float (&q1m)[9][VEC],
                                         float (&q2p)[9][VEC], float (&q2m)[9][VEC], float (&qd)[9][VEC],
                                         float (&qa)[9][VEC], float (&qb)[9][VEC], f4v &hp, f4v &hm, int s,
                                         int &es, int &er, int &eo)
{
    constexpr int a0 = S % 9, a1 = (S + 1) % 9, a2 = (S + 2) % 9, a3 = (S + 3) % 9, a4 = (S + 4) % 9,
                  a5 = (S + 5) % 9, a6 = (S + 6) % 9, a7 = (S + 7) % 9, a8 = (S + 8) % 9;
    const int r1 = C.z0 - 4 + s, r2 = r1 - 4;
    const bool in1 = r1 < C.NZr + kRadius, in_next = r1 + 4 < C.NZr + kRadius;
    const int64_t o1 = (int64_t)r1 * C.pitch + C.x;
    float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q1p[a8][j] = q1m[a8][j] = p1[j] = m1[j] = d[j] = 0.f;
    if (C.live && in_next) {
        ldv<VEC>(C.P0 + o1 + 4 * C.pitch, q1p[a8]);
        ldv<VEC>(C.M0 + o1 + 4 * C.pitch, q1m[a8]);
    }
    if (C.live && in1) {
        ldv_s<VEC>(C.P1 + o1, p1);
        ldv_s<VEC>(C.M1 + o1, m1);
        ldv_s<VEC>(C.Dp + o1, d);
    }
    const bool img1 = !GRAD && C.own_img && r1 >= C.z0 && r1 < C.z1 && r1 >= C.iz0 && r1 < C.iz1;
    if (img1) {
        ldv_s<VEC>(C.A0 + o1, qa[a4]);
        ldv_s<VEC>(C.A1 + o1, qb[a4]);
    }
    float hl[4], hr[4], ext[VEC + 8];
    float np[VEC], nm[VEC];
    f4v tm = hm;
    if constexpr (halo_ahead<VEC>()) {
        // row r1's strip-end halo was fetched one step ago; fetch row r1 + 1's
        const f4v tp = hp;
        const bool in_n1 = r1 + 1 < C.NZr + kRadius;
        hp = halo_fetch<VEC>(C.P0 + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, in_n1);
        hm = halo_fetch<VEC>(C.M0 + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, in_n1);
        halo_split(tp, C.lane, hl, hr);
    } else {
        load_halo<VEC>(C.P0 + (int64_t)r1 * C.pitch, C.xs, C.NX, C.lane, hl, hr, in1);
    }
    exchange_row<VEC>(q1p[a4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1p[a4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, q1p[a3][j], q1p[a5][j], q1p[a2][j], q1p[a6][j], q1p[a1][j], q1p[a7][j], q1p[a0][j], q1p[a8][j]);
        if constexpr (GRAD) qa[a4][j] = d[j] * lap;  // D' L p^k of row r1, used at r2
        np[j] = fmaf(d[j], lap, c2 - p1[j]);
    }
    if constexpr (halo_ahead<VEC>())
        halo_split(tm, C.lane, hl, hr);
    else
        load_halo<VEC>(C.M0 + (int64_t)r1 * C.pitch, C.xs, C.NX, C.lane, hl, hr, in1);
    exchange_row<VEC>(q1m[a4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1m[a4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, q1m[a3][j], q1m[a5][j], q1m[a2][j], q1m[a6][j], q1m[a1][j], q1m[a7][j], q1m[a0][j], q1m[a8][j]);
        nm[j] = fmaf(d[j], lap, c2 - m1[j]);
    }
    if (img1) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            qa[a4][j] = fmaf(q1p[a4][j], q1m[a4][j], qa[a4][j]);
            qb[a4][j] = fmaf(q1p[a4][j], q1p[a4][j], qb[a4][j]);
        }
    }
    // time-k terms in row r1: source re-injection into p^{k-1}, receivers into mu^k
    for (; es < C.s1end && C.ents[es].z == r1; ++es) {
        const InjEnt E = C.ents[es];
        const float sv = inj_sum(E, C.cont, C.wav);
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            if (C.reinject && E.x == C.x + j) np[j] = fmaf(d[j], sv, np[j]);
    }
    row_inject<VEC>(C.ents, C.cont, C.sig, r1, er, C.r1end, C.xs, C.lane, d, nm, C.isv, C.ihas);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        q2p[a4][j] = np[j];
        q2m[a4][j] = nm[j];
        qd[a4][j] = d[j];
    }
    if (C.own && r1 >= C.z0 && r1 < C.z1) {
        stv<VEC>(C.WP1 + o1, np);
        stv<VEC>(C.WM1 + o1, nm);
    }
    if (s >= 8 && r2 < C.z1) {
        const float hz[4] = {0.f, 0.f, 0.f, 0.f};
        const int64_t o2 = (int64_t)r2 * C.pitch + C.x;
        float vp[VEC], vm[VEC], inc2[VEC];
        exchange_row<VEC>(q2p[a0], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2p[a0][j], c2 = c + c;
            float lap =
                d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
            lap += d2(c2, q2p[a8][j], q2p[a1][j], q2p[a7][j], q2p[a2][j], q2p[a6][j], q2p[a3][j], q2p[a5][j],
                      q2p[a4][j]);
            inc2[j] = qd[a0][j] * lap;
            vp[j] = fmaf(qd[a0][j], lap, c2 - q1p[a0][j]);
        }
        exchange_row<VEC>(q2m[a0], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2m[a0][j], c2 = c + c;
            float lap =
                d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
            lap += d2(c2, q2m[a8][j], q2m[a1][j], q2m[a7][j], q2m[a2][j], q2m[a6][j], q2m[a3][j], q2m[a5][j],
                      q2m[a4][j]);
            vm[j] = fmaf(qd[a0][j], lap, c2 - q1m[a0][j]);
        }
        if (C.own) {
            stv<VEC>(C.WP2 + o2, vp);
            stv<VEC>(C.WM2 + o2, vm);
        }
        if constexpr (GRAD) {
            // source nodes of row r2 (the tile's own list): their terms of
            // steps k and k - 1, in the one-step kernel's order
            float sk[VEC], sk1[VEC];
            bool hs[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                sk[j] = sk1[j] = 0.f;
                hs[j] = false;
            }
            for (; eo < C.send && C.ents[eo].z == r2; ++eo) {
                const InjEnt E = C.ents[eo];
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    if (C.own && E.x == C.x + j) {
                        sk[j] = inj_sum(E, C.cont, C.wav);
                        sk1[j] = inj_sum(E, C.cont, C.wav - 1);
                        hs[j] = true;
                        if (C.wadj) {
                            float wsum = 0.f;
                            for (int c = E.cbeg; c < E.cend; ++c) wsum += C.cont[c].w;
                            C.wadj[(int64_t)C.k * kMaxNodes + E.slot] = wsum * q1m[a0][j];
                            C.wadj[(int64_t)(C.k - 1) * kMaxNodes + E.slot] = wsum * q2m[a0][j];
                        }
                    }
            }
            if (C.own) {
                float gg[VEC];
                ldv<VEC>(C.A0 + o2, gg);
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    gg[j] = fmaf(q1m[a0][j], qa[a0][j], gg[j]);
                    if (hs[j]) gg[j] = fmaf(q1m[a0][j], qd[a0][j] * sk[j], gg[j]);
                    gg[j] = fmaf(q2m[a0][j], inc2[j], gg[j]);
                    if (hs[j]) gg[j] = fmaf(q2m[a0][j], qd[a0][j] * sk1[j], gg[j]);
                }
                stv<VEC>(C.A0 + o2, gg);
            }
        } else if (C.own_img && r2 >= C.iz0 && r2 < C.iz1) {
            float a[VEC], bb[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                a[j] = fmaf(q2p[a0][j], q2m[a0][j], qa[a0][j]);
                bb[j] = fmaf(q2p[a0][j], q2p[a0][j], qb[a0][j]);
            }
            stv_s<VEC>(C.A0 + o2, a);
            stv_s<VEC>(C.A1 + o2, bb);
        }
    }
}

// One float per lane fits in 82 registers; asking for 5 waves per SIMD
// keeps the compiler there (it otherwise allocates 128, i.e. 4 waves).
template <int VEC, bool GRAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(VEC == 1 ? 5 : 1, 8)))
void rev2d_t2_kernel(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                     const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int k, int reinject,
                     float *__restrict__ wadj)
{
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int lane = threadIdx.x;
    Rev2Ctx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.NZr = S.L.NZr;
    C.P0 = gp(S.fld[k & 1] + S.L.org);
    C.P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    C.M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    C.M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    C.WP1 = gp(S.fld[4 + ((k + 1) & 1)] + S.L.org);
    C.WP2 = gp(S.fld[4 + (k & 1)] + S.L.org);
    C.WM1 = gp(S.fld[6 + (k & 1)] + S.L.org);
    C.WM2 = gp(S.fld[6 + ((k + 1) & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.A0 = gp(S.acc0 + S.L.org);
    C.A1 = GRAD ? nullptr : gp(S.acc1 + S.L.org);
    C.wav = S.wav + k;
    C.sig = S.sig + (int64_t)k * S.nrec;
    C.nrec = S.nrec;
    C.ents = ents;
    C.cont = cont;
    C.wadj = wadj;
    C.k = k;
    C.lane = lane;
    C.xs = T.x0;
    C.x = T.x0 + lane * VEC;
    C.z0 = T.z0;
    C.z1 = T.z1;
    C.iz0 = S.iz0;
    C.iz1 = S.iz1;
    C.s1end = T.s1end;
    C.r1end = T.r1end;
    C.send = T.send;
    __shared__ float isv[64 * VEC];
    __shared__ int ihas[64 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) ihas[lane * VEC + j] = 0;
    __syncthreads();
    C.isv = isv;
    C.ihas = ihas;
    C.live = C.x >= -kRadius && C.x < C.NX + kRadius;
    C.own = own2<VEC>(C.x, C.xs, C.NX);
    C.own_img = C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    C.reinject = reinject != 0;

    float q1p[9][VEC], q1m[9][VEC], q2p[9][VEC], q2m[9][VEC], qd[9][VEC], qa[9][VEC], qb[9][VEC];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            q1p[i][j] = q1m[i][j] = q2p[i][j] = q2m[i][j] = qd[i][j] = qa[i][j] = qb[i][j] = 0.f;
        const int r = T.z0 - 8 + i;
        if (i < 8 && C.live && r >= -kRadius) {
            ldv<VEC>(C.P0 + (int64_t)r * C.pitch + C.x, q1p[i]);
            ldv<VEC>(C.M0 + (int64_t)r * C.pitch + C.x, q1m[i]);
        }
    }
    int es = T.s1beg, er = T.r1beg, eo = T.sbeg;
    const int nstep = T.z1 - T.z0 + kZUnroll;
    // strip-end halo of the first march row (z0 - 4 >= -4: stored)
    f4v hp = halo_fetch<VEC>(C.P0 + (int64_t)(T.z0 - 4) * C.pitch, C.xs, C.NX, lane, halo_ahead<VEC>());
    f4v hm = halo_fetch<VEC>(C.M0 + (int64_t)(T.z0 - 4) * C.pitch, C.xs, C.NX, lane, halo_ahead<VEC>());
#define RTM_REV2_ROW(SS, ZZ) rev2_row<VEC, GRAD, SS>(C, q1p, q1m, q2p, q2m, qd, qa, qb, hp, hm, ZZ, es, er, eo)
    RTM_MARCH2(RTM_REV2_ROW, nstep)
#undef RTM_REV2_ROW
    // time k - 1 terms into the owned cells of p^{k-2} and mu^{k-1}
    const float *wav1 = S.wav + (k - 1);
    if (C.reinject) {
        for (int e = T.sbeg; e < T.send; ++e) {
            const InjEnt E = ents[e];
            if (owns<VEC>(E.x, C.xs, lane)) {
                const int64_t o = (int64_t)E.z * C.pitch + E.x;
                C.WP2[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav1), C.WP2[o]);
            }
        }
    }
    inject_nodes(C.WM2, C.Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)(k - 1) * S.nrec, C.pitch, C.pitch);
}

// ---------------------------------------------------------------------------
// Three steps per launch
// ---------------------------------------------------------------------------
//
// The scheme of the two-step kernels carried one step further.  A strip of
// 64 * VEC columns starting at xs overlaps its neighbours by 16 and owns the
// inner 64 * VEC - 16.  Step one (level n + 1 from n, n - 1) runs on the
// whole strip with the strip-end halo, over rows [z0 - 8, z1 + 8); step two
// runs four rows behind it and is exact on [xs + 4, xs + 64 VEC - 4) for rows
// [z0 - 4, z1 + 4); step three runs eight rows behind and is exact on the
// owned columns and rows [z0, z1).  Queue slot (S + i) % 9 holds row
// r1 - 4 + i of every queue (r1: step one's row at march step S), so step
// two's centre row r1 - 4 sits in slot S and step three's r1 - 8 in slot
// (S + 5) % 9.  Steps one and two add their sources in the march (their
// values feed the next step); step three's are added after the march by
// the owner.  Only the last two levels are stored: level n + 1 leaves the
// registers only on the rows that hold receiver nodes (modeling), so the
// launch reads two levels and D' and writes two levels once per three
// steps.  Every cell's arithmetic equals the one-step kernel's, operation
// for operation.
template <int VEC>
__device__ __forceinline__ bool own3(int x, int xs, int NX)
{
    return x >= xs + 8 && x + VEC <= xs + 64 * VEC - 8 && x < NX;
}

// Rows that exist in storage: [-4, NZr + 4).
__device__ __forceinline__ bool stored_row(int r, int NZr) { return r >= -kRadius && r < NZr + kRadius; }

// Laplacian sum of a queue's centre row: slots (c - m) and (c + m) hold
// rows -m and +m for the centre slot C (indices mod 9).
template <int VEC, int C>
__device__ __forceinline__ void lap_rows(const float (&q)[9][VEC], const float (&ext)[VEC + 8], float c2, int j,
                                         float &lap)
{
    constexpr int m1 = (C + 8) % 9, p1 = (C + 1) % 9, m2 = (C + 7) % 9, p2 = (C + 2) % 9, m3 = (C + 6) % 9,
                  p3 = (C + 3) % 9, m4 = (C + 5) % 9, p4 = (C + 4) % 9;
    lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
    lap += d2(c2, q[m1][j], q[p1][j], q[m2][j], q[p2][j], q[m3][j], q[p3][j], q[m4][j], q[p4][j]);
}

// Forward triple: levels n + 1, n + 2, n + 3 from (n, n - 1); n + 2 and
// n + 3 are stored.
template <int VEC>
struct Fwd3Ctx {
    const gfloat *pc, *pm;  // p^n, p^{n-1} (read set)
    gfloat *w2, *w3;        // p^{n+2}, p^{n+3} (write set)
    gfloat *mid;            // p^{n+1} on the receiver rows (modeling)
    const gfloat *Dp;
    const float *wav;       // wavelet from time n
    const InjEnt *ents;
    const Contrib *cont;
    int64_t pitch;
    int x, xs, NX, NZr, lane, z0, z1, e1end, e2end, m0, m1;  // [m0, m1): rows of p^{n+1} to store
    bool live, own;
};

template <int VEC, int S>
__device__ __forceinline__ void fwd3_row(const Fwd3Ctx<VEC> &C, float (&q1)[9][VEC], float (&q2)[9][VEC],
                                         float (&q3)[9][VEC], float (&qd)[9][VEC], f4v &hc, int s, int &e1,
                                         int &e2)
{
    constexpr int a0 = S % 9, a4 = (S + 4) % 9, a5 = (S + 5) % 9, a8 = (S + 8) % 9;
    const int r1 = C.z0 - 8 + s, r2 = r1 - 4, r3 = r1 - 8;
    const int64_t o1 = (int64_t)r1 * C.pitch + C.x;
    float old[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q1[a8][j] = old[j] = d[j] = 0.f;
    if (C.live && stored_row(r1 + 4, C.NZr)) ldv<VEC>(C.pc + o1 + 4 * C.pitch, q1[a8]);
    if (C.live && stored_row(r1, C.NZr)) {
        ldv<VEC>(C.pm + o1, old);
        ldv<VEC>(C.Dp + o1, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    {
        const f4v t = hc;
        hc = halo_fetch<VEC>(C.pc + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, stored_row(r1 + 1, C.NZr));
        halo_split(t, C.lane, hl, hr);
    }
    exchange_row<VEC>(q1[a4], hl, hr, ext);
    float v1[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1[a4][j], c2 = c + c;
        float lap;
        lap_rows<VEC, a4>(q1, ext, c2, j, lap);
        v1[j] = fmaf(d[j], lap, c2 - old[j]);
    }
    for (; e1 < C.e1end && C.ents[e1].z == r1; ++e1) {  // source at time n, row r1
        const InjEnt E = C.ents[e1];
        const float sv = inj_sum(E, C.cont, C.wav);
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            if (E.x == C.x + j) v1[j] = fmaf(d[j], sv, v1[j]);
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        q2[a4][j] = v1[j];
        qd[a4][j] = d[j];
    }
    if (C.own && r1 >= C.m0 && r1 < C.m1) stv<VEC>(C.mid + o1, v1);
    const float hz[4] = {0.f, 0.f, 0.f, 0.f};
    if (s >= 8 && r2 < C.z1 + 4) {
        exchange_row<VEC>(q2[a0], hz, hz, ext);
        float v2[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2[a0][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a0>(q2, ext, c2, j, lap);
            v2[j] = fmaf(qd[a0][j], lap, c2 - q1[a0][j]);
        }
        for (; e2 < C.e2end && C.ents[e2].z == r2; ++e2) {  // source at time n + 1, row r2
            const InjEnt E = C.ents[e2];
            const float sv = inj_sum(E, C.cont, C.wav + 1);
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                if (E.x == C.x + j) v2[j] = fmaf(qd[a0][j], sv, v2[j]);
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) q3[a0][j] = v2[j];
        if (C.own && r2 >= C.z0 && r2 < C.z1) stv<VEC>(C.w2 + (int64_t)r2 * C.pitch + C.x, v2);
    }
    if (s >= 16 && r3 < C.z1) {
        exchange_row<VEC>(q3[a5], hz, hz, ext);
        float v3[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q3[a5][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a5>(q3, ext, c2, j, lap);
            v3[j] = fmaf(qd[a5][j], lap, c2 - q2[a5][j]);
        }
        if (C.own) stv<VEC>(C.w3 + (int64_t)r3 * C.pitch + C.x, v3);
    }
}

// Steps n, n + 1 and n + 2 of every tile.  With receiver sampling
// (nsample > 0), the tiles also store p^{n+1} on the receiver rows into
// field 2 of the shot (a modeling job's spare slot), and the workgroups
// past the stencil slots record d^{n-2} (n >= 3: the previous launch's
// middle level, in field 6, the same buffer seen from the exchanged set),
// d^{n-1} (n > 0) and d^n from the read set.
template <int VEC>
__global__ __launch_bounds__(64) void fwd2d_t3_kernel(const ShotDev *__restrict__ shots,
                                                      const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                      const InjEnt *__restrict__ ents,
                                                      const Contrib *__restrict__ cont,
                                                      const SampleTask *__restrict__ stasks, int nsample, int n)
{
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    if (b >= nslots) {
        const int t = b - nslots, g = t / nsample;  // g = 0, 1, 2: levels n - 2, n - 1, n
        const int level = n - 2 + g;
        if (level >= 0 && (g > 0 || n >= 3))
            sample_body(shots, stasks[t - g * nsample], level, g == 0 ? 6 : (level & 1), lane);
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    Fwd3Ctx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.NZr = S.L.NZr;
    C.pc = gp(S.fld[n & 1] + S.L.org);
    C.pm = gp(S.fld[(n + 1) & 1] + S.L.org);
    C.w2 = gp(S.fld[4 + (n & 1)] + S.L.org);
    C.w3 = gp(S.fld[4 + ((n + 1) & 1)] + S.L.org);
    C.mid = nsample > 0 ? gp(S.fld[2] + S.L.org) : nullptr;
    C.m0 = nsample > 0 ? max(T.z0, S.sz0) : 0;
    C.m1 = nsample > 0 ? min(T.z1, S.sz1) : 0;
    C.Dp = gp(S.Dp + S.L.org);
    C.wav = S.wav + n;
    C.ents = ents;
    C.cont = cont;
    C.lane = lane;
    C.xs = T.x0;
    C.x = T.x0 + lane * VEC;
    C.z0 = T.z0;
    C.z1 = T.z1;
    C.e1end = T.s1end;
    C.e2end = T.s2end;
    C.live = C.x >= -kRadius && C.x < C.NX + kRadius;
    C.own = own3<VEC>(C.x, C.xs, C.NX);

    float q1[9][VEC], q2[9][VEC], q3[9][VEC], qd[9][VEC];
    // level n rows z0 - 12 .. z0 - 5 (rows above -4 do not exist: zero)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q1[i][j] = q2[i][j] = q3[i][j] = qd[i][j] = 0.f;
        const int r = T.z0 - 12 + i;
        if (i < 8 && C.live && stored_row(r, C.NZr)) ldv<VEC>(C.pc + (int64_t)r * C.pitch + C.x, q1[i]);
    }
    int e1 = T.s1beg, e2 = T.s2beg;
    // step one covers rows [z0 - 8, z1 + 8): z1 - z0 + 16 march steps,
    // rounded up to the unroll
    const int nstep = T.z1 - T.z0 + 2 * kZUnroll;
    f4v hc = halo_fetch<VEC>(C.pc + (int64_t)(T.z0 - 8) * C.pitch, C.xs, C.NX, lane, stored_row(T.z0 - 8, C.NZr));
#define RTM_FWD3_ROW(SS, ZZ) fwd3_row<VEC, SS>(C, q1, q2, q3, qd, hc, ZZ, e1, e2)
    RTM_MARCH2(RTM_FWD3_ROW, nstep)
#undef RTM_FWD3_ROW
    // Source at time n + 2 into the owned cells of level n + 3.
    const float *wav2 = S.wav + n + 2;
    for (int k = T.sbeg; k < T.send; ++k) {
        const InjEnt E = ents[k];
        if (owns<VEC>(E.x, C.xs, lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            C.w3[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav2), C.w3[o]);
        }
    }
}

// Reverse triple (imaging): steps k, k - 1 and k - 2 of the reconstruction
// and the receiver field.  All three imaging terms of a row are added at
// step two's row r2, where p^k, mu^{k+1} (step two's previous levels),
// p^{k-1}, mu^k (its centre) and the new p^{k-2}, mu^{k-1} are all in
// registers: num and den are read and written once per three steps.
template <int VEC>
struct Rev3Ctx {
    const gfloat *P0, *P1, *M0, *M1;  // p^k, p^{k+1}, mu^{k+1}, mu^{k+2} (read set)
    gfloat *WP2, *WP3, *WM2, *WM3;    // p^{k-2}, p^{k-3}, mu^{k-1}, mu^{k-2} (write set)
    const gfloat *Dp;
    gfloat *A0, *A1;                  // num, den
    const float *wav, *sig;           // wavelet and receiver signal at time k
    const InjEnt *ents;
    const Contrib *cont;
    float *isv;                       // LDS: receiver sums of one row (row_inject)
    int *ihas;
    int64_t pitch;
    int nrec;
    int x, xs, NX, NZr, lane, z0, z1, iz0, iz1, s1end, r1end, s2end, r2end;
    bool live, own, own_img, reinject;
};

template <int VEC, int S>
__device__ __forceinline__ void rev3_row(const Rev3Ctx<VEC> &C, float (&q1p)[9][VEC], float (&q1m)[9][VEC],
                                         float (&q2p)[9][VEC], float (&q2m)[9][VEC], float (&q3p)[9][VEC],
                                         float (&q3m)[9][VEC], float (&qd)[9][VEC], f4v &hp, f4v &hm, int s,
                                         int &es1, int &er1, int &es2, int &er2)
{
    constexpr int a0 = S % 9, a4 = (S + 4) % 9, a5 = (S + 5) % 9, a8 = (S + 8) % 9;
    const int r1 = C.z0 - 8 + s, r2 = r1 - 4, r3 = r1 - 8;
    const int64_t o1 = (int64_t)r1 * C.pitch + C.x, o2 = (int64_t)r2 * C.pitch + C.x;
    float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q1p[a8][j] = q1m[a8][j] = p1[j] = m1[j] = d[j] = 0.f;
    if (C.live && stored_row(r1 + 4, C.NZr)) {
        ldv<VEC>(C.P0 + o1 + 4 * C.pitch, q1p[a8]);
        ldv<VEC>(C.M0 + o1 + 4 * C.pitch, q1m[a8]);
    }
    if (C.live && stored_row(r1, C.NZr)) {
        ldv_s<VEC>(C.P1 + o1, p1);
        ldv_s<VEC>(C.M1 + o1, m1);
        ldv_s<VEC>(C.Dp + o1, d);
    }
    const bool do2 = s >= 8 && r2 < C.z1 + 4;
    const bool img = do2 && C.own_img && r2 >= C.z0 && r2 < C.z1 && r2 >= C.iz0 && r2 < C.iz1;
    float ia[VEC], ib[VEC];
    if (img) {
        ldv_s<VEC>(C.A0 + o2, ia);
        ldv_s<VEC>(C.A1 + o2, ib);
    }
    float hl[4], hr[4], ext[VEC + 8];
    float np[VEC], nm[VEC];
    const f4v tp = hp, tm = hm;
    {
        const bool en = stored_row(r1 + 1, C.NZr);
        hp = halo_fetch<VEC>(C.P0 + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, en);
        hm = halo_fetch<VEC>(C.M0 + (int64_t)(r1 + 1) * C.pitch, C.xs, C.NX, C.lane, en);
    }
    halo_split(tp, C.lane, hl, hr);
    exchange_row<VEC>(q1p[a4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1p[a4][j], c2 = c + c;
        float lap;
        lap_rows<VEC, a4>(q1p, ext, c2, j, lap);
        np[j] = fmaf(d[j], lap, c2 - p1[j]);
    }
    halo_split(tm, C.lane, hl, hr);
    exchange_row<VEC>(q1m[a4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q1m[a4][j], c2 = c + c;
        float lap;
        lap_rows<VEC, a4>(q1m, ext, c2, j, lap);
        nm[j] = fmaf(d[j], lap, c2 - m1[j]);
    }
    // time-k terms in row r1: source re-injection into p^{k-1}, receivers into mu^k
    for (; es1 < C.s1end && C.ents[es1].z == r1; ++es1) {
        const InjEnt E = C.ents[es1];
        const float sv = inj_sum(E, C.cont, C.wav);
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            if (C.reinject && E.x == C.x + j) np[j] = fmaf(d[j], sv, np[j]);
    }
    row_inject<VEC>(C.ents, C.cont, C.sig, r1, er1, C.r1end, C.xs, C.lane, d, nm, C.isv, C.ihas);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        q2p[a4][j] = np[j];
        q2m[a4][j] = nm[j];
        qd[a4][j] = d[j];
    }
    const float hz[4] = {0.f, 0.f, 0.f, 0.f};
    if (do2) {
        float vp[VEC], vm[VEC];
        exchange_row<VEC>(q2p[a0], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2p[a0][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a0>(q2p, ext, c2, j, lap);
            vp[j] = fmaf(qd[a0][j], lap, c2 - q1p[a0][j]);
        }
        exchange_row<VEC>(q2m[a0], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q2m[a0][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a0>(q2m, ext, c2, j, lap);
            vm[j] = fmaf(qd[a0][j], lap, c2 - q1m[a0][j]);
        }
        // time k - 1 terms in row r2
        for (; es2 < C.s2end && C.ents[es2].z == r2; ++es2) {
            const InjEnt E = C.ents[es2];
            const float sv = inj_sum(E, C.cont, C.wav - 1);
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                if (C.reinject && E.x == C.x + j) vp[j] = fmaf(qd[a0][j], sv, vp[j]);
        }
        row_inject<VEC>(C.ents, C.cont, C.sig - C.nrec, r2, er2, C.r2end, C.xs, C.lane, qd[a0], vm, C.isv,
                        C.ihas);
        if (C.own && r2 >= C.z0 && r2 < C.z1) {
            stv<VEC>(C.WP2 + o2, vp);
            stv<VEC>(C.WM2 + o2, vm);
        }
        if (img) {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {  // levels k, k - 1, k - 2 in turn
                ia[j] = fmaf(vp[j], vm[j], fmaf(q2p[a0][j], q2m[a0][j], fmaf(q1p[a0][j], q1m[a0][j], ia[j])));
                ib[j] = fmaf(vp[j], vp[j], fmaf(q2p[a0][j], q2p[a0][j], fmaf(q1p[a0][j], q1p[a0][j], ib[j])));
            }
            stv_s<VEC>(C.A0 + o2, ia);
            stv_s<VEC>(C.A1 + o2, ib);
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            q3p[a0][j] = vp[j];
            q3m[a0][j] = vm[j];
        }
    }
    if (s >= 16 && r3 < C.z1) {
        const int64_t o3 = (int64_t)r3 * C.pitch + C.x;
        float vp[VEC], vm[VEC];
        exchange_row<VEC>(q3p[a5], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q3p[a5][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a5>(q3p, ext, c2, j, lap);
            vp[j] = fmaf(qd[a5][j], lap, c2 - q2p[a5][j]);
        }
        exchange_row<VEC>(q3m[a5], hz, hz, ext);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q3m[a5][j], c2 = c + c;
            float lap;
            lap_rows<VEC, a5>(q3m, ext, c2, j, lap);
            vm[j] = fmaf(qd[a5][j], lap, c2 - q2m[a5][j]);
        }
        if (C.own) {
            stv<VEC>(C.WP3 + o3, vp);
            stv<VEC>(C.WM3 + o3, vm);
        }
    }
}

template <int VEC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 8)))
void rev2d_t3_kernel(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                     const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int k, int reinject)
{
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int lane = threadIdx.x;
    Rev3Ctx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.NZr = S.L.NZr;
    C.P0 = gp(S.fld[k & 1] + S.L.org);
    C.P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    C.M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    C.M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    C.WP2 = gp(S.fld[4 + (k & 1)] + S.L.org);
    C.WP3 = gp(S.fld[4 + ((k + 1) & 1)] + S.L.org);
    C.WM2 = gp(S.fld[6 + ((k + 1) & 1)] + S.L.org);
    C.WM3 = gp(S.fld[6 + (k & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.A0 = gp(S.acc0 + S.L.org);
    C.A1 = gp(S.acc1 + S.L.org);
    C.wav = S.wav + k;
    C.sig = S.sig + (int64_t)k * S.nrec;
    C.nrec = S.nrec;
    C.ents = ents;
    C.cont = cont;
    C.lane = lane;
    C.xs = T.x0;
    C.x = T.x0 + lane * VEC;
    C.z0 = T.z0;
    C.z1 = T.z1;
    C.iz0 = S.iz0;
    C.iz1 = S.iz1;
    C.s1end = T.s1end;
    C.r1end = T.r1end;
    C.s2end = T.s2end;
    C.r2end = T.r2end;
    __shared__ float isv[64 * VEC];
    __shared__ int ihas[64 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) ihas[lane * VEC + j] = 0;
    __syncthreads();
    C.isv = isv;
    C.ihas = ihas;
    C.live = C.x >= -kRadius && C.x < C.NX + kRadius;
    C.own = own3<VEC>(C.x, C.xs, C.NX);
    C.own_img = C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    C.reinject = reinject != 0;

    float q1p[9][VEC], q1m[9][VEC], q2p[9][VEC], q2m[9][VEC], q3p[9][VEC], q3m[9][VEC], qd[9][VEC];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j)
            q1p[i][j] = q1m[i][j] = q2p[i][j] = q2m[i][j] = q3p[i][j] = q3m[i][j] = qd[i][j] = 0.f;
        const int r = T.z0 - 12 + i;
        if (i < 8 && C.live && stored_row(r, C.NZr)) {
            ldv<VEC>(C.P0 + (int64_t)r * C.pitch + C.x, q1p[i]);
            ldv<VEC>(C.M0 + (int64_t)r * C.pitch + C.x, q1m[i]);
        }
    }
    int es1 = T.s1beg, er1 = T.r1beg, es2 = T.s2beg, er2 = T.r2beg;
    const int nstep = T.z1 - T.z0 + 2 * kZUnroll;
    const bool en0 = stored_row(T.z0 - 8, C.NZr);
    f4v hp = halo_fetch<VEC>(C.P0 + (int64_t)(T.z0 - 8) * C.pitch, C.xs, C.NX, lane, en0);
    f4v hm = halo_fetch<VEC>(C.M0 + (int64_t)(T.z0 - 8) * C.pitch, C.xs, C.NX, lane, en0);
#define RTM_REV3_ROW(SS, ZZ) rev3_row<VEC, SS>(C, q1p, q1m, q2p, q2m, q3p, q3m, qd, hp, hm, ZZ, es1, er1, es2, er2)
    RTM_MARCH2(RTM_REV3_ROW, nstep)
#undef RTM_REV3_ROW
    // time k - 2 terms into the owned cells of p^{k-3} and mu^{k-2}
    const float *wav2 = S.wav + (k - 2);
    if (C.reinject) {
        for (int e = T.sbeg; e < T.send; ++e) {
            const InjEnt E = ents[e];
            if (owns<VEC>(E.x, C.xs, lane)) {
                const int64_t o = (int64_t)E.z * C.pitch + E.x;
                C.WP3[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav2), C.WP3[o]);
            }
        }
    }
    inject_nodes(C.WM3, C.Dp, ents, T.rbeg, T.rend, cont, S.sig + (int64_t)(k - 2) * S.nrec, C.pitch, C.pitch);
}

// ---------------------------------------------------------------------------
// Persistent passes: one launch for all time steps of a pass
// ---------------------------------------------------------------------------
//
// A grid small enough to be resident as a whole (sized from the occupancy
// of the kernel) walks the pass's work items (tiles, and in modeling the
// receiver sampling tasks) step after step: workgroup b takes items b,
// b + G, b + 2G, ... of every step.  The steps of different shots are not
// tied to each other: an item of shot s at step r waits only until the
// counter of shot s shows all of that shot's items of step r - 1 done
// (r * items(s) completions), so a shot with little work runs ahead of a
// larger one.  One wave per workgroup: after an item the wave makes its
// stores visible to the whole GPU (agent-scope release fence, which also
// writes them back from this XCD's L2) and lane 0 increments the counter;
// a waiting wave's lane 0 reads the counter, and once it suffices the wave
// takes an agent-scope acquire fence (dropping stale L1/L2 lines) before
// touching the fields.  Every wait is bounded: after `limit` ticks of the
// constant 100 MHz clock, or as soon as another workgroup has given up, the
// waiting workgroup sets *status and returns, so a grid that cannot make
// progress (not all workgroups resident) still ends.

// Waits until *cnt >= target (lane 0 polls); false if the pass was abandoned.
__device__ __forceinline__ bool persist_wait(unsigned *cnt, unsigned target, unsigned *status, uint64_t limit,
                                             int lane)
{
    int ok = 1;
    if (lane == 0) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                wall_clock64() - t0 > limit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

// Publishes the item just done: this wave's stores, then the count.
__device__ __forceinline__ void persist_done(unsigned *cnt, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Forward steps n0 .. n0 + nsteps - 1 (fwd2d_kernel's step, one strip per
// workgroup), with the sampling tasks of each step when stasks != nullptr.
template <int VEC>
__global__ __launch_bounds__(64) void fwd2d_persist_kernel(const ShotDev *__restrict__ shots,
                                                           const Tile2D *__restrict__ tiles,
                                                           const PItem *__restrict__ items, int nitems,
                                                           const int *__restrict__ shot_items,
                                                           const InjEnt *__restrict__ ents,
                                                           const Contrib *__restrict__ cont,
                                                           const SampleTask *__restrict__ stasks, int n0, int nsteps,
                                                           unsigned *cnt, unsigned *status, uint64_t limit)
{
    const int lane = threadIdx.x & 63;
    __shared__ EdgeRing<1> ring;
    for (int r = 0; r < nsteps; ++r) {
        const int n = n0 + r;
        for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
            const PItem it = items[i];
            if (!persist_wait(cnt + it.shot, (unsigned)r * (unsigned)shot_items[it.shot], status, limit, lane)) return;
            if (it.idx >= 0) {
                fwd2d_tile<VEC, 1>(shots, tiles, it.idx, ents, cont, n, 0, lane, ring);
            } else {
                sample_body(shots, stasks[-1 - it.idx], n, n & 1, lane);
            }
            persist_done(cnt + it.shot, lane);
        }
    }
}

// Reverse steps k0, k0 - 1, ..., k0 - nsteps + 1 (rev2d_kernel's step).
template <int VEC, bool GRAD>
__global__ __launch_bounds__(64) void rev2d_persist_kernel(const ShotDev *__restrict__ shots, const Tile2D *__restrict__ tiles,
                          const PItem *__restrict__ items, int nitems, const int *__restrict__ shot_items,
                          const InjEnt *__restrict__ ents, const Contrib *__restrict__ cont, int k0, int nsteps,
                          int reinject, float *__restrict__ wadj, unsigned *cnt, unsigned *status, uint64_t limit)
{
    const int lane = threadIdx.x & 63;
    __shared__ EdgeRing<1> ring_p, ring_m;
    for (int r = 0; r < nsteps; ++r) {
        const int k = k0 - r;
        for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
            const PItem it = items[i];
            if (!persist_wait(cnt + it.shot, (unsigned)r * (unsigned)shot_items[it.shot], status, limit, lane)) return;
            rev2d_tile<VEC, GRAD, 1>(shots, tiles, it.idx, ents, cont, k, reinject, wadj, 0, lane, ring_p, ring_m);
            persist_done(cnt + it.shot, lane);
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

// Workgroups of a persistent launch: at most what the GPU holds resident at
// once (occupancy of the kernel times the compute units), at most nitems;
// and the bounded wait in ticks of the constant clock.
template <class K>
hipError_t persist_grid(K kernel, int nitems, double wait_ms, int *grid, uint64_t *limit)
{
    int dev = 0, cus = 0, per_cu = 0, khz = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0)) != hipSuccess) return e;
    if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
    const int64_t g = std::min<int64_t>((int64_t)per_cu * cus, nitems);
    *grid = (int)std::max<int64_t>(g, 1);
    *limit = (uint64_t)((double)(khz > 0 ? khz : 100000) * wait_ms);
    return hipSuccess;
}

template <int V>
hipError_t fwd2d_persist_launch(const ShotDev *shots, const Tile2D *tiles, const PItem *items, int nitems,
                                const int *shot_items, const InjEnt *ents, const Contrib *cont,
                                const SampleTask *stasks, int n0, int nsteps, unsigned *cnt, unsigned *status,
                                double wait_ms, hipStream_t st)
{
    int grid = 0;
    uint64_t limit = 0;
    hipError_t e = persist_grid(fwd2d_persist_kernel<V>, nitems, wait_ms, &grid, &limit);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd2d_persist_kernel<V>), dim3(grid), dim3(64), 0, st, shots, tiles, items, nitems,
                       shot_items, ents, cont, stasks, n0, nsteps, cnt, status, limit);
    return hipGetLastError();
}

template <int V, bool G>
hipError_t rev2d_persist_launch(const ShotDev *shots, const Tile2D *tiles, const PItem *items, int nitems,
                                const int *shot_items, const InjEnt *ents, const Contrib *cont, int k0, int nsteps,
                                int reinject, float *wadj, unsigned *cnt, unsigned *status, double wait_ms,
                                hipStream_t st)
{
    int grid = 0;
    uint64_t limit = 0;
    hipError_t e = persist_grid(rev2d_persist_kernel<V, G>, nitems, wait_ms, &grid, &limit);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rev2d_persist_kernel<V, G>), dim3(grid), dim3(64), 0, st, shots, tiles, items, nitems,
                       shot_items, ents, cont, k0, nsteps, reinject, wadj, cnt, status, limit);
    return hipGetLastError();
}

hipError_t launch_fwd2d_persist(int vec, const ShotDev *shots, const Tile2D *tiles, const PItem *items, int nitems,
                                const int *shot_items, const InjEnt *ents, const Contrib *cont,
                                const SampleTask *stasks, int n0, int nsteps, unsigned *cnt, unsigned *status,
                                double wait_ms, hipStream_t st)
{
    if (nitems < 1 || nsteps < 1) return hipSuccess;
    switch (vec) {
    case 1: return fwd2d_persist_launch<1>(shots, tiles, items, nitems, shot_items, ents, cont, stasks, n0, nsteps, cnt,
                                           status, wait_ms, st);
    case 2: return fwd2d_persist_launch<2>(shots, tiles, items, nitems, shot_items, ents, cont, stasks, n0, nsteps, cnt,
                                           status, wait_ms, st);
    case 4: return fwd2d_persist_launch<4>(shots, tiles, items, nitems, shot_items, ents, cont, stasks, n0, nsteps, cnt,
                                           status, wait_ms, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rev2d_persist(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, const PItem *items,
                                int nitems, const int *shot_items, const InjEnt *ents, const Contrib *cont, int k0,
                                int nsteps, int reinject, float *wadj, unsigned *cnt, unsigned *status,
                                double wait_ms, hipStream_t st)
{
    if (nitems < 1 || nsteps < 1) return hipSuccess;
#define RTM_REVP(V, G) \
    rev2d_persist_launch<V, G>(shots, tiles, items, nitems, shot_items, ents, cont, k0, nsteps, reinject, wadj, cnt, \
                               status, wait_ms, st)
    switch (vec * 2 + (grad ? 1 : 0)) {
    case 2: return RTM_REVP(1, false);
    case 3: return RTM_REVP(1, true);
    case 4: return RTM_REVP(2, false);
    case 5: return RTM_REVP(2, true);
    case 8: return RTM_REVP(4, false);
    case 9: return RTM_REVP(4, true);
    default: return hipErrorInvalidValue;
    }
#undef RTM_REVP
}

hipError_t launch_fwd2d(int vec, int tx, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st)
{
    dim3 grid(nslots + (nsample + tx - 1) / tx), block(64 * tx);
#define RTM_FWD2D(V, X) \
    hipLaunchKernelGGL((fwd2d_kernel<V, X>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n)
#define RTM_FWD2D_X(V)                              \
    switch (tx) {                                   \
    case 1: RTM_FWD2D(V, 1); break;                 \
    case 2: RTM_FWD2D(V, 2); break;                 \
    case 4: RTM_FWD2D(V, 4); break;                 \
    default: return hipErrorInvalidValue;           \
    }
    switch (vec) {
    case 1: RTM_FWD2D_X(1); break;
    case 2: RTM_FWD2D_X(2); break;
    case 4: RTM_FWD2D_X(4); break;
    default: return hipErrorInvalidValue;
    }
#undef RTM_FWD2D_X
#undef RTM_FWD2D
    return hipGetLastError();
}

hipError_t launch_rev2d(int vec, int tx, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles,
                        int nslots, const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj,
                        hipStream_t st)
{
    dim3 grid(nslots), block(64 * tx);
#define RTM_REV2D(V, G, X) \
    hipLaunchKernelGGL((rev2d_kernel<V, G, X>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject, wadj)
#define RTM_REV2D_X(V, G)                           \
    switch (tx) {                                   \
    case 1: RTM_REV2D(V, G, 1); break;              \
    case 2: RTM_REV2D(V, G, 2); break;              \
    case 4: RTM_REV2D(V, G, 4); break;              \
    default: return hipErrorInvalidValue;           \
    }
    if (grad) {
        switch (vec) {
        case 1: RTM_REV2D_X(1, true); break;
        case 2: RTM_REV2D_X(2, true); break;
        case 4: RTM_REV2D_X(4, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (vec) {
        case 1: RTM_REV2D_X(1, false); break;
        case 2: RTM_REV2D_X(2, false); break;
        case 4: RTM_REV2D_X(4, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef RTM_REV2D_X
#undef RTM_REV2D
    return hipGetLastError();
}

hipError_t launch_recv2d(int vec, int tx, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                         const InjEnt *ents, const Contrib *cont, int k, const float *snap, hipStream_t st)
{
    dim3 grid(nslots), block(64 * tx);
#define RTM_RECV2D(V, X)                                                                                             \
    if (snap)                                                                                                        \
        hipLaunchKernelGGL((recv2d_kernel<V, X, true>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, \
                           snap);                                                                                    \
    else                                                                                                             \
        hipLaunchKernelGGL((recv2d_kernel<V, X, false>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, \
                           k, snap)
#define RTM_RECV2D_X(V)                             \
    switch (tx) {                                   \
    case 1: RTM_RECV2D(V, 1); break;                \
    case 2: RTM_RECV2D(V, 2); break;                \
    case 4: RTM_RECV2D(V, 4); break;                \
    default: return hipErrorInvalidValue;           \
    }
    switch (vec) {
    case 1: RTM_RECV2D_X(1); break;
    case 2: RTM_RECV2D_X(2); break;
    case 4: RTM_RECV2D_X(4); break;
    default: return hipErrorInvalidValue;
    }
#undef RTM_RECV2D_X
#undef RTM_RECV2D
    return hipGetLastError();
}

hipError_t launch_fwd2d_t2(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                           hipStream_t st)
{
    dim3 grid(nslots + 2 * nsample), block(64);
    switch (vec) {
    case 1: hipLaunchKernelGGL(fwd2d_t2_kernel<1>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    case 2: hipLaunchKernelGGL(fwd2d_t2_kernel<2>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    case 4: hipLaunchKernelGGL(fwd2d_t2_kernel<4>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rev2d_t2(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st)
{
    dim3 grid(nslots), block(64);
#define RTM_REV2T2(V, G) \
    hipLaunchKernelGGL((rev2d_t2_kernel<V, G>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject, wadj)
    switch (vec * 2 + (grad ? 1 : 0)) {
    case 2: RTM_REV2T2(1, false); break;
    case 3: RTM_REV2T2(1, true); break;
    case 4: RTM_REV2T2(2, false); break;
    case 5: RTM_REV2T2(2, true); break;
    case 8: RTM_REV2T2(4, false); break;
    case 9: RTM_REV2T2(4, true); break;
    default: return hipErrorInvalidValue;
    }
#undef RTM_REV2T2
    return hipGetLastError();
}

hipError_t launch_fwd2d_t3(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                           hipStream_t st)
{
    dim3 grid(nslots + 3 * nsample), block(64);
    switch (vec) {
    case 1: hipLaunchKernelGGL(fwd2d_t3_kernel<1>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    case 2: hipLaunchKernelGGL(fwd2d_t3_kernel<2>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    case 4: hipLaunchKernelGGL(fwd2d_t3_kernel<4>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, nsample, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rev2d_t3(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                           const InjEnt *ents, const Contrib *cont, int k, int reinject, hipStream_t st)
{
    dim3 grid(nslots), block(64);
    switch (vec) {
    case 1: hipLaunchKernelGGL(rev2d_t3_kernel<1>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject); break;
    case 2: hipLaunchKernelGGL(rev2d_t3_kernel<2>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject); break;
    case 4: hipLaunchKernelGGL(rev2d_t3_kernel<4>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rtm
