// Device helpers shared by the 2-D and 3-D propagation kernels: global
// address-space views, vector loads and stores, DPP lane shifts, the
// 8th-order second difference, strip halos and injection sums.
#pragma once

#include "common.h"

namespace rtm {
namespace {

constexpr float kC1 = 1.6f;
constexpr float kC2 = -0.2f;
constexpr float kC3 = 8.0f / 315.0f;
constexpr float kC4 = -1.0f / 560.0f;

// Global-address-space views: plain global loads and stores instead of
// flat ones (which would also count against the scalar-memory wait).
typedef __attribute__((address_space(1))) float gfloat;
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f2v gf2v;
typedef __attribute__((address_space(1))) f4v gf4v;
__device__ __forceinline__ gfloat *gp(float *p) { return (gfloat *)p; }
__device__ __forceinline__ const gfloat *gp(const float *p) { return (const gfloat *)p; }

__device__ __forceinline__ float dpp_shr1(float old, float src)
{
    // wave_shr:1 - lane i receives lane i-1; lane 0 keeps `old`.
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x138, 0xf,
                                                      0xf, false));
}

__device__ __forceinline__ float dpp_shl1(float old, float src)
{
    // wave_shl:1 - lane i receives lane i+1; lane 63 keeps `old`.
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x130, 0xf,
                                                      0xf, false));
}

template <int VEC>
__device__ __forceinline__ void ldv(const gfloat *p, float (&v)[VEC])
{
    if constexpr (VEC == 4) {
        const f4v t = *(const gf4v *)p;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (VEC == 2) {
        const f2v t = *(const gf2v *)p;
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = *p;
    }
}

// Loads and stores of the arrays a launch streams through once (the _s
// forms mark those call sites; they are the plain accesses).
template <int VEC>
__device__ __forceinline__ void ldv_s(const gfloat *p, float (&v)[VEC])
{
    ldv<VEC>(p, v);
}

template <int VEC>
__device__ __forceinline__ void stv(gfloat *p, const float (&v)[VEC]);

template <int VEC>
__device__ __forceinline__ void stv_s(gfloat *p, const float (&v)[VEC])
{
    stv<VEC>(p, v);
}

template <int VEC>
__device__ __forceinline__ void stv(gfloat *p, const float (&v)[VEC])
{
    if constexpr (VEC == 4) {
        *(gf4v *)p = f4v{v[0], v[1], v[2], v[3]};
    } else if constexpr (VEC == 2) {
        *(gf2v *)p = f2v{v[0], v[1]};
    } else {
        *p = v[0];
    }
}

// Unscaled 8th-order second difference along one direction: c2 = 2 p_i,
// (m_k, p_k) the neighbours at distance k.
__device__ __forceinline__ float d2(float c2, float m1, float p1, float m2, float p2, float m3, float p3, float m4,
                                    float p4)
{
    float s = kC1 * ((p1 + m1) - c2);
    s = fmaf(kC2, (p2 + m2) - c2, s);
    s = fmaf(kC3, (p3 + m3) - c2, s);
    s = fmaf(kC4, (p4 + m4) - c2, s);
    return s;
}

// Row of 4 + VEC + 4 values around the lane's VEC centre cells, built from
// the neighbouring lanes by DPP shifts.  hl / hr are the halo floats at the
// strip ends (meaningful in lanes 0 and 63 only).
template <int VEC>
__device__ __forceinline__ void exchange_row(const float (&c)[VEC], const float (&hl)[4], const float (&hr)[4],
                                             float (&ext)[VEC + 8])
{
    constexpr int K = 4 / VEC;
#pragma unroll
    for (int j = 0; j < VEC; ++j) ext[4 + j] = c[j];
    float L[VEC], Rr[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        L[j] = c[j];
        Rr[j] = c[j];
    }
#pragma unroll
    for (int k = 1; k <= K; ++k) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            L[j] = dpp_shr1(hl[4 - k * VEC + j], L[j]);
            Rr[j] = dpp_shl1(hr[(k - 1) * VEC + j], Rr[j]);
            ext[4 - k * VEC + j] = L[j];
            ext[4 + VEC + (k - 1) * VEC + j] = Rr[j];
        }
    }
}

// Strip-end halo of one row: lane 0 loads the 4 cells left of the strip,
// lane 63 the 4 cells right of it (zeros past the stored columns); one load
// instruction for both.
template <int VEC>
__device__ __forceinline__ void load_halo(const gfloat *row, int x0, int NX, int lane, float (&hl)[4],
                                          float (&hr)[4], bool enable = true)
{
    // enable = false (a row outside the stored grid): no load, zero halo.
    const int xr = x0 + 64 * VEC;
    const bool left = enable && lane == 0, right = enable && lane == 63 && xr < NX + kRadius;
    f4v t = f4v{0.f, 0.f, 0.f, 0.f};
    if (left || right) t = *(const gf4v *)(row + (left ? x0 - 4 : xr));
    hl[0] = left ? t.x : 0.f; hl[1] = left ? t.y : 0.f; hl[2] = left ? t.z : 0.f; hl[3] = left ? t.w : 0.f;
    hr[0] = right ? t.x : 0.f; hr[1] = right ? t.y : 0.f; hr[2] = right ? t.z : 0.f; hr[3] = right ? t.w : 0.f;
}

// The same halo in two parts, so that the load can be issued rows before
// its use: halo_fetch loads the 4 cells beyond the strip's left end (lane 0)
// or right end (lane 63) of a row; halo_split hands them out as hl / hr.
template <int VEC>
__device__ __forceinline__ f4v halo_fetch(const gfloat *row, int x0, int NX, int lane, bool enable)
{
    const int xr = x0 + 64 * VEC;
    const bool left = enable && lane == 0, right = enable && lane == 63 && xr < NX + kRadius;
    f4v t = f4v{0.f, 0.f, 0.f, 0.f};
    if (left || right) t = *(const gf4v *)(row + (left ? x0 - 4 : xr));
    return t;
}

// exchange_row reads hl only in lane 0 (the lane a right shift leaves
// without a source) and hr only in lane 63, which are the lanes that loaded
// the left and the right halo: both are the fetched values as they are, with
// no per-lane selection and no second set of registers.
__device__ __forceinline__ void halo_split(f4v t, int lane, float (&hl)[4], float (&hr)[4])
{
    (void)lane;
    hl[0] = hr[0] = t.x;
    hl[1] = hr[1] = t.y;
    hl[2] = hr[2] = t.z;
    hl[3] = hr[3] = t.w;
}

// Strip-end halo of one row for a wave inside a workgroup of strips: only
// the workgroup's outer ends (do_left in the first wave, do_right in the
// last) are loaded from memory; inner ends come from the edge ring.
template <int VEC>
__device__ __forceinline__ void load_halo_outer(const gfloat *row, int x0, int NX, int lane, bool do_left,
                                                bool do_right, float (&hl)[4], float (&hr)[4])
{
    const int xr = x0 + 64 * VEC;
    const bool left = do_left && lane == 0, right = do_right && lane == 63 && xr < NX + kRadius;
    f4v t = f4v{0.f, 0.f, 0.f, 0.f};
    if (left || right) t = *(const gf4v *)(row + (left ? x0 - 4 : xr));
    hl[0] = left ? t.x : 0.f; hl[1] = left ? t.y : 0.f; hl[2] = left ? t.z : 0.f; hl[3] = left ? t.w : 0.f;
    hr[0] = right ? t.x : 0.f; hr[1] = right ? t.y : 0.f; hr[2] = right ? t.z : 0.f; hr[3] = right ? t.w : 0.f;
}

// Edge ring of a workgroup of TX strip wavefronts (LDS): slot s, wave w
// holds the 4 leftmost (side 0) and 4 rightmost (side 1) cells of one row of
// the wave's strip.  A row is published when it enters the register queue
// and read when it reaches the queue centre, four rows later.
template <int TX>
struct EdgeRing {
    float v[9][TX][2][4];
};

template <int VEC, int TX>
__device__ __forceinline__ void ring_put(EdgeRing<TX> &R, int s, int w, int lane, const float (&c)[VEC])
{
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const int cl = lane * VEC + j;
        if (cl < 4) R.v[s][w][0][cl] = c[j];
        const int cr = cl - (64 * VEC - 4);
        if (cr >= 0) R.v[s][w][1][cr] = c[j];
    }
}

template <int TX>
__device__ __forceinline__ void ring_get(const EdgeRing<TX> &R, int s, int w, int lane, float (&hl)[4],
                                         float (&hr)[4])
{
    if (lane == 0 && w > 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) hl[k] = R.v[s][w - 1][1][k];
    }
    if (lane == 63 && w < TX - 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) hr[k] = R.v[s][w + 1][0][k];
    }
}

// Receivers [r0, r0 + 64) of one shot: d[n][r] = sum_q w_q p^n[node_q],
// with p^n held by field `slot` of the shot.
__device__ __forceinline__ void sample_body(const ShotDev *__restrict__ shots, SampleTask task, int n, int slot,
                                            int lane)
{
    const ShotDev &S = shots[task.shot];
    int r = task.r0 + lane;
    if (r >= S.nrec) return;
    const gfloat *p = gp(S.fld[slot] + S.L.org);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kMaxNodes; ++q) {
        float w = S.rw[r * kMaxNodes + q];
        int off = S.rnode[r * kMaxNodes + q];
        s = fmaf(w, p[off], s);
    }
    gp(S.rec_out)[(int64_t)n * S.nrec + r] = s;
}

// Weighted signal sum of one injection entry.
__device__ __forceinline__ float inj_sum(const InjEnt &E, const Contrib *__restrict__ cont, const float *sig)
{
    float s = 0.f;
    for (int c = E.cbeg; c < E.cend; ++c) s = fmaf(cont[c].w, sig[cont[c].idx], s);
    return s;
}

// Receiver term of a reverse step at the tile's receiver nodes
// ents[beg, end): f += Dp * (weighted signal sum).  Every node lies in the
// tile and appears once, so the workgroup's threads take the nodes in
// parallel, after a barrier that orders the march's stores of f before
// these read-modify-writes (one thread per node would otherwise walk the
// whole list: at a receiver line with a receiver per column that serial
// walk outlasts the march).  plane == pitch and y == 0 in 2-D.
__device__ __forceinline__ void inject_nodes(gfloat *f, const gfloat *Dp, const InjEnt *__restrict__ ents, int beg,
                                             int end, const Contrib *__restrict__ cont, const float *sig,
                                             int64_t plane, int64_t pitch)
{
    __syncthreads();
    for (int e = beg + (int)threadIdx.x; e < end; e += (int)blockDim.x) {
        const InjEnt E = ents[e];
        const int64_t o = (int64_t)E.z * plane + (int64_t)E.y * pitch + E.x;
        f[o] = fmaf(Dp[o], inj_sum(E, cont, sig), f[o]);
    }
}

// Inside a wavefront's march: adds Dp * (weighted signal sum) into v at the
// lane's VEC cells for every entry ents[e ..) of row r (entries sorted by
// row, each column at most once per row; e advances past them).  The lanes
// take up to 64 entries at a time and hand each sum to the owning lane
// through LDS (sv, has: 64 * VEC slots, has zero on entry), instead of every
// lane walking the list.  The workgroup is this one wavefront, and e and r
// are uniform, so the barriers are reached by every lane.
template <int VEC>
__device__ __forceinline__ void row_inject(const InjEnt *ents, const Contrib *__restrict__ cont, const float *sig,
                                           int r, int &e, int eend, int xs, int lane, const float (&d)[VEC],
                                           float (&v)[VEC], float *sv, int *has)
{
    if (e >= eend || ents[e].z != r) return;
    while (true) {
        const int i = e + lane;
        const bool mine = i < eend && ents[i].z == r;
        const unsigned long long m = __ballot(mine);
        if (mine) {
            const InjEnt E = ents[i];
            const int col = E.x - xs;
            sv[col] = inj_sum(E, cont, sig);
            has[col] = 1;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const int c = lane * VEC + j;
            if (has[c]) {
                v[j] = fmaf(d[j], sv[c], v[j]);
                has[c] = 0;
            }
        }
        __syncthreads();
        const int n = __popcll(m);
        e += n;
        if (n < 64) break;
    }
}

// Does this lane own padded column x of a strip starting at x0?
template <int VEC>
__device__ __forceinline__ bool owns(int x, int x0, int lane)
{
    return x >= x0 + lane * VEC && x < x0 + (lane + 1) * VEC;
}

// Imaging from a stored source level (migration with wavefield storage,
// Algorithm 2): for the lane's cells x .. x + VEC - 1 of padded row (z, y),
// num += p^k mu^{k+1} and den += (p^k)^2, p^k read from the dense interior
// snapshot [nz][ny][nx] of that level.  The caller checks that (z, y) is an
// interior row and the lane overlaps the interior columns; cells outside
// them add zero.
struct SnapImg {
    const float *snap;
    int64_t nxi, nyi;
    int ix0, ix1, iy0, iz0;
};

template <int VEC>
__device__ __forceinline__ void snap_image(const SnapImg &I, gfloat *A0, gfloat *A1, int64_t o, int z, int y, int x,
                                           const float (&mu)[VEC])
{
    const int64_t row = ((int64_t)(z - I.iz0) * I.nyi + (y - I.iy0)) * I.nxi;
    float s[VEC], a[VEC], b[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const int xx = x + j;
        s[j] = (xx >= I.ix0 && xx < I.ix1) ? I.snap[row + (xx - I.ix0)] : 0.f;
    }
    ldv<VEC>(A0 + o, a);
    ldv<VEC>(A1 + o, b);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        a[j] = fmaf(s[j], mu[j], a[j]);
        b[j] = fmaf(s[j], s[j], b[j]);
    }
    stv<VEC>(A0 + o, a);
    stv<VEC>(A1 + o, b);
}

}  // namespace
}  // namespace rtm
