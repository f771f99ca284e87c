/* Drives every entry point of the FP64 oracle on tiny 2-D and 3-D grids
 * (off-grid source and receivers, band options, storage decimation), for a
 * run under AddressSanitizer and UBSan.  Prints "ALL OK" when every call
 * returned 0 and every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_rbc_pad_ex(int, long, long, long, int, const float *, uint64_t, float, unsigned, double, float *);
int orc_pad_adjoint_ex(int, long, long, long, int, const float *, uint64_t, float, unsigned, double, const double *,
                       double *);
int orc_taper(int, double, float *);
int orc_laplacian(int, long, long, long, double, const double *, double *);
int orc_model_shot(int, long, long, long, int, double, const float *, double, int, const double *, const double *, int,
                   const double *, const double *, double *, double *, double *);
int orc_rtm_shot(int, long, long, long, int, double, const float *, double, int, const double *, const double *, int,
                 const double *, const double *, int, double, double *, double *, double *, double *, double *, int,
                 double *, double *);
int orc_rtm_storage_shot(int, long, long, long, int, double, const float *, double, int, const double *, const double *,
                         int, const double *, const double *, int, int, double, double *, double *, double *);

static int finite_all(const double *x, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static int run(int ndim)
{
    const long nx = 9, ny = ndim == 3 ? 7 : 1, nz = 8;
    const int nb = 3, nt = 40, nrec = 3;
    const long NX = nx + 2 * nb, NY = ndim == 3 ? ny + 2 * nb : 1, NZ = nz + 2 * nb;
    const long ni = nx * ny * nz, np = NX * NY * NZ;
    int bad = 0;
    float *v = malloc(sizeof(float) * ni), *vp = malloc(sizeof(float) * np), c[8];
    for (long i = 0; i < ni; ++i) v[i] = 1800.0f + 3.0f * (float)(i % 97);
    bad |= orc_taper(nb, 0.5, c);
    bad |= orc_rbc_pad_ex(ndim, nx, ny, nz, nb, v, 11, 0.0f, 3u, 0.5, vp);
    double *gp = malloc(sizeof(double) * np), *gi = malloc(sizeof(double) * ni), *lap = malloc(sizeof(double) * np);
    for (long i = 0; i < np; ++i) gp[i] = sin(0.1 * (double)i);
    bad |= orc_pad_adjoint_ex(ndim, nx, ny, nz, nb, v, 11, 0.0f, 3u, 0.5, gp, gi);
    bad |= orc_laplacian(ndim, NX, NY, NZ, 10.0, gp, lap);
    bad |= orc_rbc_pad_ex(ndim, nx, ny, nz, nb, v, 11, 0.0f, 0u, 0.0, vp);
    double w[40], src[3] = {4.3, ndim == 3 ? 3.5 : 0.0, 2.25}, rec[9] = {0.0, 0.0, 1.5, 8.0, ndim == 3 ? 6.0 : 0.0, 7.0,
                                                                         3.25, ndim == 3 ? 2.5 : 0.0, 0.0};
    for (int n = 0; n < nt; ++n) w[n] = sin(0.3 * n) * exp(-0.01 * n * n);
    double *tr = malloc(sizeof(double) * nrec * (nt + 1)), *pl = malloc(sizeof(double) * np),
           *pp = malloc(sizeof(double) * np);
    bad |= orc_model_shot(ndim, nx, ny, nz, nb, 10.0, vp, 1e-3, nt, w, src, nrec, rec, NULL, tr, pl, pp);
    bad |= !finite_all(tr, nrec * (nt + 1));
    double *num = malloc(sizeof(double) * ni), *den = malloc(sizeof(double) * ni), *img = malloc(sizeof(double) * ni),
           *grad = malloc(sizeof(double) * np), *wadj = malloc(sizeof(double) * nt), *sp = malloc(sizeof(double) * np),
           *sm = malloc(sizeof(double) * np);
    bad |= orc_rtm_shot(ndim, nx, ny, nz, nb, 10.0, vp, 1e-3, nt, w, src, nrec, rec, tr, 1, 1e-3, num, den, img, grad,
                        wadj, nt / 2, sp, sm);
    bad |= !finite_all(img, ni) || !finite_all(grad, np) || !finite_all(wadj, nt);
    bad |= orc_rtm_storage_shot(ndim, nx, ny, nz, nb, 10.0, vp, 1e-3, nt, w, src, nrec, rec, tr, 3, 1, 1e-3, num, den,
                                img);
    bad |= !finite_all(img, ni);
    free(v); free(vp); free(gp); free(gi); free(lap); free(tr); free(pl); free(pp);
    free(num); free(den); free(img); free(grad); free(wadj); free(sp); free(sm);
    return bad;
}

int main(void)
{
    int bad = run(2) | run(3);
    printf(bad ? "FAILED\n" : "ALL OK\n");
    return bad;
}
