/*
 * FP64 CPU oracle for random-boundary reverse time migration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this file: it exists so that tests/, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation written from the paper
 * (Barbosa & Coutinho, "Seismic Modeling and Migration with Random Boundaries
 * on the NEC SX-Aurora TSUBASA", arXiv 2204.03380).  It shares no code,
 * header, constant or helper with the HIP library.
 *
 * Conventions:
 *  - Grids: interior extents nx, ny, nz (ny = 1 in 2-D), spacing h, padded
 *    with nb random-boundary cells on every face.  Padded arrays are stored
 *    [NZ][NY][NX], x fastest, with NX = nx + 2nb, NZ = nz + 2nb and
 *    NY = ny + 2nb in 3-D (1 in 2-D).
 *  - Outside the padded grid the wavefield is zero: the Dirichlet condition
 *    p = 0 on the domain boundary stated with Eq. (1) and Eq. (6).
 *  - Positions are in interior grid units: (x, y, z), 0-based, relative to
 *    interior cell (0, 0, 0); y is ignored in 2-D.
 *  - Time: wavelet samples w[0..nt-1]; traces d[r][0..nt] (nt + 1 samples
 *    per receiver, Sec. 3), with d^0 = 0 from the zero initial state.
 *
 * Every loop below follows the definition it cites; nothing is blocked,
 * fused or reordered beyond what the definition itself states.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>

/* ------------------------------------------------------------------ */
/* Grid bookkeeping                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int ndim;
    long nx, ny, nz; /* interior */
    int nb;
    long NX, NY, NZ; /* padded */
    double h;
} og_grid;

static int og_make(og_grid *g, int ndim, long nx, long ny, long nz, int nb, double h)
{
    if (ndim != 2 && ndim != 3) return -1;
    if (nx < 1 || nz < 1 || nb < 0) return -1;
    if (ndim == 2) ny = 1;
    if (ny < 1) return -1;
    g->ndim = ndim;
    g->nx = nx; g->ny = ny; g->nz = nz; g->nb = nb; g->h = h;
    g->NX = nx + 2L * nb;
    g->NZ = nz + 2L * nb;
    g->NY = (ndim == 3) ? ny + 2L * nb : 1;
    return 0;
}

static long og_cells(const og_grid *g) { return g->NX * g->NY * g->NZ; }

static long og_index(const og_grid *g, long z, long y, long x)
{
    return (z * g->NY + y) * g->NX + x;
}

/* Value of a padded field, zero outside the padded grid (Dirichlet). */
static double og_at(const og_grid *g, const double *p, long z, long y, long x)
{
    if (x < 0 || x >= g->NX || y < 0 || y >= g->NY || z < 0 || z >= g->NZ) return 0.0;
    return p[og_index(g, z, y, x)];
}

/* ------------------------------------------------------------------ */
/* Random boundary velocities (Sec. "Wavefield Reconstruction", Eqs.   */
/* (4)-(5) context): uniform factors in [0.7, 1.3) times the nearest   */
/* interior edge velocity, capped to keep the scheme stable.           */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the (k+1)-th output of a
 * generator whose state starts at `seed` and advances by the golden-ratio
 * increment, passed through the 64-bit finaliser. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static long og_clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Band options (the paper's setup, Sec. "Wavefield Reconstruction" and the
 * model description of the 2-D and 3-D tests). */
#define ORC_RBC_TAPER 1u        /* scale band velocities by c_i, Eqs. (4)-(5) */
#define ORC_RBC_FREE_SURFACE 2u /* top band: v = 0 (p stays 0 above the surface) */

/* Taper coefficient of band depth i = 1 .. nb (i = 1 touches the interior):
 * c_i = alpha g(i) + (1 - alpha) h(i) with Eq. (4) g(i) = (nb - i)/(nb - 1)
 * and Eq. (5) h(i) = exp(-120 (i - 1)^2 / (nb - 1)^2), evaluated in double
 * and rounded once to FP32; nb = 1 gives c_1 = 1.  For alpha in [0, 1] the
 * value lies between h and g. */
static float og_taper(int nb, int i, double alpha)
{
    if (nb <= 1) return 1.0f;
    double x = (double)i, n1 = (double)(nb - 1);
    double g = ((double)nb - x) / n1;
    double hh = exp(-120.0 * (x - 1.0) * (x - 1.0) / (n1 * n1));
    return (float)(alpha * g + (1.0 - alpha) * hh);
}

/* Distance of padded cell coordinate a (interior at [0, n)) from the
 * interior along one axis: 0 inside. */
static long og_depth(long a, long n) { return a < 0 ? -a : (a >= n ? a - n + 1 : 0); }

/* Random factor of band cell j: f_j = fmaf(0.6f, u_j, 0.7f), u_j the top 24
 * bits of SplitMix64(seed, j) scaled by 2^-24. */
static float og_rbc_factor(uint64_t seed, long j)
{
    uint64_t r = orc_splitmix64(seed, (uint64_t)j);
    float u = (float)(r >> 40) * (1.0f / 16777216.0f);
    return fmaf(0.6f, u, 0.7f);
}

static float og_vmax(const float *v, long n)
{
    float m = v[0];
    for (long i = 0; i < n; ++i)
        if (v[i] > m) m = v[i];
    return m;
}

/* Random boundary with options.  Interior: v_pad = v_int.  Band cell j at
 * depth i (the largest per-axis distance from the interior) with edge value
 * v_edge (the nearest interior cell):
 *   default:   fminf(f_j * v_edge, v_cap)
 *   TAPER:     fminf(c_i * (f_j * v_edge), v_cap)
 *   FREE_SURFACE and the cell lies above the interior (z < 0): 0.
 * All values are FP32 by definition and match the GPU bit for bit.
 * v_cap <= 0 selects the interior maximum.  Returns 0, or -1 on bad args. */
int orc_rbc_pad_ex(int ndim, long nx, long ny, long nz, int nb, const float *v_int, uint64_t seed, float v_cap,
                   unsigned flags, double alpha, float *v_pad)
{
    og_grid g;
    if (og_make(&g, ndim, nx, ny, nz, nb, 1.0) != 0 || !v_int || !v_pad) return -1;
    if ((flags & ORC_RBC_TAPER) && !(alpha >= 0.0 && alpha <= 1.0)) return -1;
    if (!(v_cap > 0.0f)) v_cap = og_vmax(v_int, g.nx * g.ny * g.nz);
    for (long z = 0; z < g.NZ; ++z)
        for (long y = 0; y < g.NY; ++y)
            for (long x = 0; x < g.NX; ++x) {
                long iz = z - nb, ix = x - nb, iy = (ndim == 3) ? y - nb : 0;
                long d = og_depth(ix, g.nx), dz = og_depth(iz, g.nz), dy = ndim == 3 ? og_depth(iy, g.ny) : 0;
                if (dz > d) d = dz;
                if (dy > d) d = dy;
                long ez = og_clampl(iz, 0, g.nz - 1);
                long ey = og_clampl(iy, 0, g.ny - 1);
                long ex = og_clampl(ix, 0, g.nx - 1);
                float v_edge = v_int[(ez * g.ny + ey) * g.nx + ex];
                long j = og_index(&g, z, y, x);
                if (d == 0) {
                    v_pad[j] = v_edge;
                } else if ((flags & ORC_RBC_FREE_SURFACE) && iz < 0) {
                    v_pad[j] = 0.0f;
                } else {
                    float v = og_rbc_factor(seed, j) * v_edge;
                    if (flags & ORC_RBC_TAPER) v = og_taper(nb, (int)d, alpha) * v;
                    v_pad[j] = fminf(v, v_cap);
                }
            }
    return 0;
}

int orc_rbc_pad(int ndim, long nx, long ny, long nz, int nb, const float *v_int,
                uint64_t seed, float v_cap, float *v_pad)
{
    return orc_rbc_pad_ex(ndim, nx, ny, nz, nb, v_int, seed, v_cap, 0u, 0.0, v_pad);
}

/* Adjoint of the padding with respect to v_int, with the random factors,
 * the taper and v_cap held fixed: interior cells pass their gradient
 * through; a band cell adds (c_i) f_j times its gradient to its edge cell
 * unless it was capped (value >= v_cap, where the derivative is zero); a
 * free-surface cell (v = 0 whatever v_int) adds nothing. */
int orc_pad_adjoint_ex(int ndim, long nx, long ny, long nz, int nb, const float *v_int, uint64_t seed, float v_cap,
                       unsigned flags, double alpha, const double *grad_pad, double *grad_int)
{
    og_grid g;
    if (og_make(&g, ndim, nx, ny, nz, nb, 1.0) != 0 || !v_int || !grad_pad || !grad_int) return -1;
    if ((flags & ORC_RBC_TAPER) && !(alpha >= 0.0 && alpha <= 1.0)) return -1;
    if (!(v_cap > 0.0f)) v_cap = og_vmax(v_int, g.nx * g.ny * g.nz);
    for (long i = 0; i < g.nx * g.ny * g.nz; ++i) grad_int[i] = 0.0;
    for (long z = 0; z < g.NZ; ++z)
        for (long y = 0; y < g.NY; ++y)
            for (long x = 0; x < g.NX; ++x) {
                long iz = z - nb, ix = x - nb, iy = (ndim == 3) ? y - nb : 0;
                long d = og_depth(ix, g.nx), dz = og_depth(iz, g.nz), dy = ndim == 3 ? og_depth(iy, g.ny) : 0;
                if (dz > d) d = dz;
                if (dy > d) d = dy;
                long ez = og_clampl(iz, 0, g.nz - 1);
                long ey = og_clampl(iy, 0, g.ny - 1);
                long ex = og_clampl(ix, 0, g.nx - 1);
                long e = (ez * g.ny + ey) * g.nx + ex;
                long j = og_index(&g, z, y, x);
                if (d == 0) {
                    grad_int[e] += grad_pad[j];
                } else if ((flags & ORC_RBC_FREE_SURFACE) && iz < 0) {
                    /* constant zero */
                } else {
                    float f = og_rbc_factor(seed, j);
                    float v = f * v_int[e];
                    double scale = (double)f;
                    if (flags & ORC_RBC_TAPER) {
                        float c = og_taper(nb, (int)d, alpha);
                        v = c * v;
                        scale *= (double)c;
                    }
                    if (v < v_cap) grad_int[e] += scale * grad_pad[j];
                }
            }
    return 0;
}

int orc_pad_adjoint(int ndim, long nx, long ny, long nz, int nb, const float *v_int,
                    uint64_t seed, float v_cap, const double *grad_pad, double *grad_int)
{
    return orc_pad_adjoint_ex(ndim, nx, ny, nz, nb, v_int, seed, v_cap, 0u, 0.0, grad_pad, grad_int);
}

/* Taper table for the pins: c[i - 1] for i = 1 .. nb. */
int orc_taper(int nb, double alpha, float *c)
{
    if (nb < 1 || !c || !(alpha >= 0.0 && alpha <= 1.0)) return -1;
    for (int i = 1; i <= nb; ++i) c[i - 1] = og_taper(nb, i, alpha);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Spatial operator (Sec. 3: 8th order in space)                       */
/* ------------------------------------------------------------------ */

/* Centred 9-point second-derivative weights of 8th order: the unique
 * symmetric set with sum_m 2 c_m m^(2k) = 2 for k = 1 and 0 for k = 2..4. */
static const double OG_C0 = -205.0 / 72.0;
static const double OG_CM[5] = {0.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

/* out = L_h p: the sum over axes of the 1-D second-difference operator,
 * divided by h^2, with p = 0 outside the padded grid.  Cells at least four
 * cells from every face read their neighbours directly; the others through
 * og_at, which supplies the zeros outside.  Both evaluate the same sum in
 * the same order. */
static void og_laplacian(const og_grid *g, const double *p, double *out)
{
    const double inv_h2 = 1.0 / (g->h * g->h);
    const long sy = g->NX, sz = g->NX * g->NY;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < g->NZ; ++z)
        for (long y = 0; y < g->NY; ++y)
            for (long x = 0; x < g->NX; ++x) {
                const int inner = x >= 4 && x < g->NX - 4 && z >= 4 && z < g->NZ - 4 &&
                                  (g->ndim == 2 || (y >= 4 && y < g->NY - 4));
                if (inner) {
                    const long j = og_index(g, z, y, x);
                    double s = g->ndim * OG_C0 * p[j];
                    for (int m = 1; m <= 4; ++m) {
                        s += OG_CM[m] * (p[j + m] + p[j - m]);
                        s += OG_CM[m] * (p[j + m * sz] + p[j - m * sz]);
                        if (g->ndim == 3) s += OG_CM[m] * (p[j + m * sy] + p[j - m * sy]);
                    }
                    out[j] = s * inv_h2;
                    continue;
                }
                double s = g->ndim * OG_C0 * og_at(g, p, z, y, x);
                for (int m = 1; m <= 4; ++m) {
                    s += OG_CM[m] * (og_at(g, p, z, y, x + m) + og_at(g, p, z, y, x - m));
                    s += OG_CM[m] * (og_at(g, p, z + m, y, x) + og_at(g, p, z - m, y, x));
                    if (g->ndim == 3)
                        s += OG_CM[m] * (og_at(g, p, z, y + m, x) + og_at(g, p, z, y - m, x));
                }
                out[og_index(g, z, y, x)] = s * inv_h2;
            }
}

/* Exported for the consistency pins: the padded grid is given directly. */
int orc_laplacian(int ndim, long NX, long NY, long NZ, double h, const double *p, double *out)
{
    og_grid g;
    if (og_make(&g, ndim, NX, NY, NZ, 0, h) != 0 || !p || !out) return -1;
    og_laplacian(&g, p, out);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Point operators: multilinear interpolation weights                  */
/* ------------------------------------------------------------------ */

#define OG_MAXNODE 8

typedef struct {
    int n;
    long idx[OG_MAXNODE];
    double w[OG_MAXNODE];
} og_point;

/* Nodes and weights of the multilinear interpolant at an interior position
 * (x, y, z); zero weights are dropped, so an on-grid point is one node of
 * weight 1.  Returns -1 if the point lies outside the interior. */
static int og_point_make(const og_grid *g, const double pos[3], og_point *pt)
{
    double q[3] = {pos[0], g->ndim == 3 ? pos[1] : 0.0, pos[2]};
    long n_ax[3] = {g->nx, g->ny, g->nz};
    long i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        if (!(q[a] >= 0.0 && q[a] <= (double)(n_ax[a] - 1))) return -1;
        i0[a] = (long)floor(q[a]);
        fr[a] = q[a] - (double)i0[a];
    }
    pt->n = 0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double w = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) *
                           (cz ? fr[2] : 1.0 - fr[2]);
                if (w == 0.0) continue;
                long px = i0[0] + cx + g->nb;
                long py = (g->ndim == 3) ? i0[1] + cy + g->nb : 0;
                long pz = i0[2] + cz + g->nb;
                pt->idx[pt->n] = og_index(g, pz, py, px);
                pt->w[pt->n] = w;
                pt->n++;
            }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Modeling: Eq. (1) advanced by the explicit scheme of Sec. 3,        */
/* Algorithm 1 (one shot).                                             */
/* ------------------------------------------------------------------ */

/* Checks shared by the shot routines; fills the source and receiver
 * operators.  Returns 0, -1 (bad arguments) or -3 (position outside). */
static int og_setup(og_grid *g, int ndim, long nx, long ny, long nz, int nb, double h, int nt,
                    const double *src, int nrec, const double *rec, og_point *sp, og_point **rp)
{
    if (og_make(g, ndim, nx, ny, nz, nb, h) != 0 || nt < 1 || nrec < 0 || !src) return -1;
    if (nrec > 0 && !rec) return -1;
    if (og_point_make(g, src, sp) != 0) return -3;
    *rp = (og_point *)calloc(nrec > 0 ? (size_t)nrec : 1, sizeof(og_point));
    for (int r = 0; r < nrec; ++r)
        if (og_point_make(g, rec + 3L * r, &(*rp)[r]) != 0) {
            free(*rp);
            *rp = NULL;
            return -3;
        }
    return 0;
}

/* One leapfrog step of the second-order time discretisation:
 *   pn1 = 2 p - pm1 + D (L_h p + B w_n + m p)
 * with D = (v dt)^2 and B the source interpolant scaled by h^-d (a discrete
 * point source).  pn1 may alias pm1. */
static void og_step(const og_grid *g, const double *D, const double *p, const double *pm1,
                    double *pn1, double *lap, const og_point *sp, double wn, const double *m)
{
    og_laplacian(g, p, lap);
    double hd = pow(g->h, g->ndim);
    for (int k = 0; k < sp->n; ++k) lap[sp->idx[k]] += sp->w[k] / hd * wn;
    long n = og_cells(g);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double rhs = lap[i] + (m ? m[i] * p[i] : 0.0);
        pn1[i] = 2.0 * p[i] - pm1[i] + D[i] * rhs;
    }
}

static double og_sample(const og_point *rp, const double *p)
{
    double s = 0.0;
    for (int k = 0; k < rp->n; ++k) s += rp->w[k] * p[rp->idx[k]];
    return s;
}

/* Forward modeling of one shot (Algorithm 1; Eq. (1) with zero initial
 * state).  traces[r*(nt+1) + n] = R_r p^n for n = 0..nt.  Optionally
 * returns the last two states p^nt and p^(nt-1) (padded), the two panels
 * the reconstruction starts from.  m (padded, nullable) adds m*p to the
 * right-hand side; it is used only by the image identity pin.
 * Returns 0, -1 (bad arguments) or -3 (position outside the interior). */
int orc_model_shot(int ndim, long nx, long ny, long nz, int nb, double h, const float *v_pad,
                   double dt, int nt, const double *w, const double *src, int nrec,
                   const double *rec, const double *m, double *traces, double *p_last,
                   double *p_prev)
{
    og_grid g;
    og_point sp, *rp = NULL;
    int rc = og_setup(&g, ndim, nx, ny, nz, nb, h, nt, src, nrec, rec, &sp, &rp);
    if (rc != 0) return rc;
    if (!v_pad || !w || (nrec > 0 && !traces)) {
        free(rp);
        return -1;
    }
    long n = og_cells(&g);
    double *D = (double *)malloc(sizeof(double) * n);
    double *a = (double *)calloc(n, sizeof(double)); /* p^n */
    double *b = (double *)calloc(n, sizeof(double)); /* p^(n-1), then p^(n+1) */
    double *lap = (double *)malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) D[i] = ((double)v_pad[i] * dt) * ((double)v_pad[i] * dt);

    for (int r = 0; r < nrec; ++r) traces[(long)r * (nt + 1)] = og_sample(&rp[r], a);
    for (int it = 0; it < nt; ++it) {
        og_step(&g, D, a, b, b, lap, &sp, w[it], m);
        double *t = a;
        a = b;
        b = t; /* a = p^(it+1), b = p^it */
        for (int r = 0; r < nrec; ++r)
            traces[(long)r * (nt + 1) + it + 1] = og_sample(&rp[r], a);
    }
    if (p_last) memcpy(p_last, a, sizeof(double) * n);
    if (p_prev) memcpy(p_prev, b, sizeof(double) * n);
    free(D);
    free(a);
    free(b);
    free(lap);
    free(rp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Migration with wavefield reconstruction: Algorithm 3, Eqs. (2),     */
/* (3) and (6).                                                        */
/* ------------------------------------------------------------------ */

/* One shot of RTM with random boundaries and reconstruction.
 *
 * Forward pass (Algorithm 3, source wavefield): as orc_model_shot, keeping
 * only the last two panels p^nt, p^(nt-1).
 * Reverse pass, k = nt-1 down to 0, carrying both
 *   - the reconstructed source wavefield (Eq. (6)), stepping the same
 *     scheme backwards: p^(k-1) = 2 p^k - p^(k+1) + D (L_h p^k + B w^k).
 *     With reinject = 0 the source term is dropped, as Eq. (6) is written;
 *   - the receiver wavefield (Eq. (2)) as the exact discrete adjoint of the
 *     forward scheme: mu^k = 2 mu^(k+1) - mu^(k+2) + D L_h mu^(k+1) + D R^T g^k,
 *     started from mu^(nt+1) = mu^(nt+2) = 0;
 * and accumulating the two integrals of Eq. (3) with the pairing
 * p^k <-> mu^(k+1):  num += p^k mu^(k+1),  den += (p^k)^2.
 * image = num / (den + eps_rel * max(den)) on the interior crop.
 *
 * g[r*(nt+1) + n] holds the data injected at the receivers (the recorded
 * seismogram for migration, or an upstream gradient).
 * Optional outputs (nullable):
 *   num, den, image  interior-sized;
 *   grad_pad         padded: dJ/dv = 2 G / (v^3 dt^2) with
 *                    G = sum_k mu^(k+1) (p^(k+1) - 2 p^k + p^(k-1));
 *   w_adj[n]         = <B, mu^(n+1)>, n = 0..nt-1 (adjoint wrt the wavelet);
 *   snap_p, snap_mu  padded reconstructed p^snap_k and mu^snap_k,
 *                    for 0 <= snap_k <= nt-2 (snap_k < 0: none).
 * Returns 0, -1 or -3. */
static int og_rtm(int ndim, long nx, long ny, long nz, int nb, double h, const float *v_pad,
                  double dt, int nt, const double *w, const double *src, int nrec,
                  const double *rec, const double *g_in, int reinject, double eps_rel,
                  double *num_out, double *den_out, double *image, double *grad_pad,
                  double *w_adj, int snap_k, double *snap_p, double *snap_mu,
                  const double *start_last, const double *start_prev)
{
    og_grid g;
    og_point sp, *rp = NULL;
    int rc = og_setup(&g, ndim, nx, ny, nz, nb, h, nt, src, nrec, rec, &sp, &rp);
    if (rc != 0) return rc;
    if (!v_pad || !w || (nrec > 0 && !g_in) || (snap_k >= 0 && snap_k > nt - 2)) {
        free(rp);
        return -1;
    }
    long n = og_cells(&g);
    double hd = pow(g.h, g.ndim);
    double *D = (double *)malloc(sizeof(double) * n);
    double *pa = (double *)calloc(n, sizeof(double));
    double *pb = (double *)calloc(n, sizeof(double));
    double *ma = (double *)calloc(n, sizeof(double));
    double *mb = (double *)calloc(n, sizeof(double));
    double *lap = (double *)malloc(sizeof(double) * n);
    double *lapm = (double *)malloc(sizeof(double) * n);
    double *num = (double *)calloc(n, sizeof(double));
    double *den = (double *)calloc(n, sizeof(double));
    double *G = (double *)calloc(n, sizeof(double));
    double *src_term = (double *)calloc(n, sizeof(double));
    for (long i = 0; i < n; ++i) D[i] = ((double)v_pad[i] * dt) * ((double)v_pad[i] * dt);

    /* Forward: pa = p^n, pb = p^(n-1); or the two panels given. */
    if (start_last && start_prev) {
        memcpy(pa, start_last, sizeof(double) * n);
        memcpy(pb, start_prev, sizeof(double) * n);
    } else {
        for (int it = 0; it < nt; ++it) {
            og_step(&g, D, pa, pb, pb, lap, &sp, w[it], NULL);
            double *t = pa;
            pa = pb;
            pb = t;
        }
    }
    /* Now pa = p^nt, pb = p^(nt-1).  Rename for the reverse pass:
     * P1 = p^(k+1), P0 = p^k; M1 = mu^(k+2), M0 = mu^(k+1). */
    double *P1 = pa, *P0 = pb, *M1 = mb, *M0 = ma;
    for (long i = 0; i < n; ++i) M1[i] = 0.0; /* mu^(nt+1) */
    for (long i = 0; i < n; ++i) M0[i] = 0.0; /* mu^nt = D R^T g^nt */
    for (int r = 0; r < nrec; ++r)
        for (int k = 0; k < rp[r].n; ++k)
            M0[rp[r].idx[k]] += D[rp[r].idx[k]] * rp[r].w[k] * g_in[(long)r * (nt + 1) + nt];

    for (int k = nt - 1; k >= 0; --k) {
        /* Imaging condition, Eq. (3): p^k paired with mu^(k+1). */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            num[i] += P0[i] * M0[i];
            den[i] += P0[i] * P0[i];
        }
        if (w_adj) {
            double s = 0.0;
            for (int q = 0; q < sp.n; ++q) s += sp.w[q] / hd * M0[sp.idx[q]];
            w_adj[k] = s;
        }
        /* Reconstruction, Eq. (6).  d2 = D (L_h p^k + B w^k) is the second
         * time difference of the forward field at step k; the gradient pairs
         * it with mu^(k+1).  The reconstruction re-injects the source term
         * unless reinject = 0 (Eq. (6) as written, with a zero right side). */
        og_laplacian(&g, P0, lap);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) src_term[i] = 0.0;
        for (int q = 0; q < sp.n; ++q) src_term[sp.idx[q]] += sp.w[q] / hd * w[k];
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            double d2 = D[i] * (lap[i] + src_term[i]);
            G[i] += M0[i] * d2;
            double step = reinject ? d2 : D[i] * lap[i];
            P1[i] = 2.0 * P0[i] - P1[i] + step;
        }
        /* Receiver wavefield, Eq. (2) as the discrete adjoint. */
        og_laplacian(&g, M0, lapm);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) M1[i] = 2.0 * M0[i] - M1[i] + D[i] * lapm[i];
        for (int r = 0; r < nrec; ++r)
            for (int q = 0; q < rp[r].n; ++q)
                M1[rp[r].idx[q]] += D[rp[r].idx[q]] * rp[r].w[q] * g_in[(long)r * (nt + 1) + k];
        /* P1 now holds p^(k-1) and M1 holds mu^k: rotate. */
        double *t = P1;
        P1 = P0;
        P0 = t;
        t = M1;
        M1 = M0;
        M0 = t;
        if (snap_k >= 0 && k - 1 == snap_k && snap_p) memcpy(snap_p, P0, sizeof(double) * n);
        if (snap_k >= 0 && k == snap_k && snap_mu) memcpy(snap_mu, M0, sizeof(double) * n);
    }

    /* Interior crop and normalisation (Eq. (3)). */
    double dmax = 0.0;
    for (long z = 0; z < g.nz; ++z)
        for (long y = 0; y < g.ny; ++y)
            for (long x = 0; x < g.nx; ++x) {
                long j = og_index(&g, z + nb, g.ndim == 3 ? y + nb : 0, x + nb);
                if (den[j] > dmax) dmax = den[j];
            }
    for (long z = 0; z < g.nz; ++z)
        for (long y = 0; y < g.ny; ++y)
            for (long x = 0; x < g.nx; ++x) {
                long j = og_index(&g, z + nb, g.ndim == 3 ? y + nb : 0, x + nb);
                long o = (z * g.ny + y) * g.nx + x;
                if (num_out) num_out[o] = num[j];
                if (den_out) den_out[o] = den[j];
                if (image) image[o] = num[j] / (den[j] + eps_rel * dmax);
            }
    if (grad_pad)
        for (long i = 0; i < n; ++i) {
            /* dJ/dv = 2 v dt^2 dJ/dD: zero where v = 0 (a free-surface band) */
            double v = (double)v_pad[i];
            grad_pad[i] = v == 0.0 ? 0.0 : 2.0 * G[i] / (v * v * v * dt * dt);
        }
    free(D);
    free(pa);
    free(pb);
    free(ma);
    free(mb);
    free(lap);
    free(lapm);
    free(num);
    free(den);
    free(G);
    free(src_term);
    free(rp);
    return 0;
}

int orc_rtm_shot(int ndim, long nx, long ny, long nz, int nb, double h, const float *v_pad,
                 double dt, int nt, const double *w, const double *src, int nrec,
                 const double *rec, const double *g_in, int reinject, double eps_rel,
                 double *num_out, double *den_out, double *image, double *grad_pad,
                 double *w_adj, int snap_k, double *snap_p, double *snap_mu)
{
    return og_rtm(ndim, nx, ny, nz, nb, h, v_pad, dt, nt, w, src, nrec, rec, g_in, reinject, eps_rel,
                  num_out, den_out, image, grad_pad, w_adj, snap_k, snap_p, snap_mu, NULL, NULL);
}

/* orc_rtm_shot with the forward pass replaced by its result: p_last = p^nt
 * and p_prev = p^(nt-1) (padded, as orc_model_shot returns them), from
 * which the reverse pass starts.  Equal to orc_rtm_shot when the panels
 * come from orc_model_shot on the same inputs. */
int orc_rtm_shot_panels(int ndim, long nx, long ny, long nz, int nb, double h, const float *v_pad,
                        double dt, int nt, const double *w, const double *src, int nrec,
                        const double *rec, const double *g_in, int reinject, double eps_rel,
                        double *num_out, double *den_out, double *image, const double *p_last,
                        const double *p_prev)
{
    if (!p_last || !p_prev) return -1;
    return og_rtm(ndim, nx, ny, nz, nb, h, v_pad, dt, nt, w, src, nrec, rec, g_in, reinject, eps_rel,
                  num_out, den_out, image, NULL, NULL, -1, NULL, NULL, p_last, p_prev);
}

/* ------------------------------------------------------------------ */
/* Migration with wavefield storage: Algorithm 2, with the source      */
/* wavefield kept only every `stride` steps (the decimation of         */
/* Eq. (7)).                                                           */
/* ------------------------------------------------------------------ */

/* One shot of RTM that stores the source wavefield instead of
 * reconstructing it.
 * Forward pass: the scheme of orc_model_shot; p^k is kept for every
 * k in [0, nt-1] with k = phase (mod stride).
 * Reverse pass, k = nt-1 down to 0: only the receiver wavefield (Eq. (2),
 * the same discrete adjoint as orc_rtm_shot); at every kept k the imaging
 * sums of Eq. (3) take the stored p^k with mu^(k+1):
 *     num += p^k mu^(k+1),  den += (p^k)^2.
 * image = num / (den + eps_rel * max(den)) on the interior crop.
 * With stride = 1 the sums equal those of the reconstruction.
 * Returns 0, -1 or -3. */
int orc_rtm_storage_shot(int ndim, long nx, long ny, long nz, int nb, double h, const float *v_pad,
                         double dt, int nt, const double *w, const double *src, int nrec,
                         const double *rec, const double *g_in, int stride, int phase, double eps_rel,
                         double *num_out, double *den_out, double *image)
{
    og_grid g;
    og_point sp, *rp = NULL;
    int rc = og_setup(&g, ndim, nx, ny, nz, nb, h, nt, src, nrec, rec, &sp, &rp);
    if (rc != 0) return rc;
    if (!v_pad || !w || (nrec > 0 && !g_in) || stride < 1 || phase < 0 || phase >= stride) {
        free(rp);
        return -1;
    }
    long n = og_cells(&g);
    long nkeep = 0;
    for (int k = phase; k < nt; k += stride) ++nkeep;
    double *D = (double *)malloc(sizeof(double) * n);
    double *a = (double *)calloc(n, sizeof(double));
    double *b = (double *)calloc(n, sizeof(double));
    double *lap = (double *)malloc(sizeof(double) * n);
    double *store = (double *)calloc((size_t)(nkeep > 0 ? nkeep : 1) * n, sizeof(double));
    for (long i = 0; i < n; ++i) D[i] = ((double)v_pad[i] * dt) * ((double)v_pad[i] * dt);

    /* Forward: a = p^it before the step.  Keep p^it for kept it. */
    for (int it = 0; it < nt; ++it) {
        if (it >= phase && (it - phase) % stride == 0)
            memcpy(store + (size_t)((it - phase) / stride) * n, a, sizeof(double) * n);
        og_step(&g, D, a, b, b, lap, &sp, w[it], NULL);
        double *t = a;
        a = b;
        b = t;
    }
    /* Reverse: M0 = mu^(k+1), M1 = mu^(k+2). */
    double *M0 = a, *M1 = b;
    double *num = (double *)calloc(n, sizeof(double));
    double *den = (double *)calloc(n, sizeof(double));
    for (long i = 0; i < n; ++i) M1[i] = 0.0;
    for (long i = 0; i < n; ++i) M0[i] = 0.0;
    for (int r = 0; r < nrec; ++r)
        for (int q = 0; q < rp[r].n; ++q)
            M0[rp[r].idx[q]] += D[rp[r].idx[q]] * rp[r].w[q] * g_in[(long)r * (nt + 1) + nt];
    for (int k = nt - 1; k >= 0; --k) {
        if (k >= phase && (k - phase) % stride == 0) {
            const double *pk = store + (size_t)((k - phase) / stride) * n;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                num[i] += pk[i] * M0[i];
                den[i] += pk[i] * pk[i];
            }
        }
        og_laplacian(&g, M0, lap);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) M1[i] = 2.0 * M0[i] - M1[i] + D[i] * lap[i];
        for (int r = 0; r < nrec; ++r)
            for (int q = 0; q < rp[r].n; ++q)
                M1[rp[r].idx[q]] += D[rp[r].idx[q]] * rp[r].w[q] * g_in[(long)r * (nt + 1) + k];
        double *t = M1;
        M1 = M0;
        M0 = t;
    }
    double dmax = 0.0;
    for (long z = 0; z < g.nz; ++z)
        for (long y = 0; y < g.ny; ++y)
            for (long x = 0; x < g.nx; ++x) {
                long j = og_index(&g, z + nb, g.ndim == 3 ? y + nb : 0, x + nb);
                if (den[j] > dmax) dmax = den[j];
            }
    for (long z = 0; z < g.nz; ++z)
        for (long y = 0; y < g.ny; ++y)
            for (long x = 0; x < g.nx; ++x) {
                long j = og_index(&g, z + nb, g.ndim == 3 ? y + nb : 0, x + nb);
                long o = (z * g.ny + y) * g.nx + x;
                if (num_out) num_out[o] = num[j];
                if (den_out) den_out[o] = den[j];
                if (image) image[o] = num[j] / (den[j] + eps_rel * dmax);
            }
    free(D);
    free(a);
    free(b);
    free(lap);
    free(store);
    free(num);
    free(den);
    free(rp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Run environment of the timed baseline (no arithmetic)               */
/* ------------------------------------------------------------------ */

/* Threads of the parallel loops from now on (n >= 1); returns the count in
 * effect afterwards. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* The calling thread's SSE control state: bit 0 set if denormal results are
 * flushed to zero (FTZ), bit 1 if denormal inputs are read as zero (DAZ). */
int orc_fp_env(void)
{
    const unsigned csr = _mm_getcsr();
    return ((csr >> 15) & 1u) | (((csr >> 6) & 1u) << 1);
}
