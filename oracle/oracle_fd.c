/*
 * FP64 reference time loop for 2-D constant-density acoustic modelling.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU path is
 * checked against. It is built with gcc and is loaded only by the test suite,
 * by the smoke check and by the CPU-baseline leg of the benchmark; the product
 * path never calls it. It shares no code with the HIP library.
 *
 * What it computes (paper, Testing approach section: finite differences of
 * second order in time and eighth order in space, damping-layer absorbing
 * boundary of nbpml points, Ricker source, one receiver per surface sample):
 *
 *   PDE   m (u_tt + d u_t) - Lap u = f,      m = 1/v^2
 *   scheme (centred second difference in time, centred first difference for
 *   the damping term, a = d*dt/2):
 *     u^{n+1} = [ 2 u^n - (1-a) u^{n-1} + (v dt)^2 (Lap_h u^n + f^n) ] / (1+a)
 *   for n = 0 .. nt-2, with u^0 = u^{-1} = 0 unless initial fields are given.
 *   Lap_h u = sum_{k=-4..4} w[|k|] ( u(I+k,J)/dz^2 + u(I,J+k)/dx^2 ), with
 *   u = 0 outside the grid (homogeneous Dirichlet beyond the absorbing layer).
 *   f^n = wavelet[n] * sw / (dz*dx) at each source point (a discrete delta).
 *   traces[n][r] = sum_k rw_k u^n(rI_k, rJ_k) over the points of receiver r,
 *   for n = 0 .. nt-1.
 *
 * Plain triple loop, no blocking, no reordering. The caller supplies the
 * stencil weights, the velocity and the damping coefficient on the padded
 * grid, so that every convention is decided in readable Python.
 */
#include <stdlib.h>
#include <string.h>

#define IDX(I, J) ((size_t)(I) * (size_t)Nx + (size_t)(J))

int oracle_forward_run(
    int Nz, int Nx, double dz, double dx,
    const double *w,          /* [5] second-derivative weights w[0..4]          */
    const double *vel,        /* [Nz][Nx] velocity on the padded grid (m/s)      */
    const double *damp,       /* [Nz][Nx] damping coefficient d (1/s)            */
    double dt, int nt,
    const double *wavelet,    /* [nt] source time function, or NULL              */
    int nsp, const int *sI, const int *sJ, const double *sw,   /* source points  */
    int nrec, int nrp, const int *rI, const int *rJ, const double *rw,
    const int *rid,           /* [nrp] receiver index of each sampling point     */
    double *traces,           /* [nt][nrec] output, or NULL                      */
    const double *u0,         /* u^0 or NULL (zero)                              */
    const double *um1,        /* u^{-1} or NULL (zero)                           */
    double *ufinal)           /* u^{nt-1} output, or NULL                        */
{
    size_t N = (size_t)Nz * (size_t)Nx;
    double *u = calloc(N, sizeof(double));
    double *uprev = calloc(N, sizeof(double));
    double *unext = calloc(N, sizeof(double));
    if (!u || !uprev || !unext) {
        free(u); free(uprev); free(unext);
        return -1;
    }
    if (u0) memcpy(u, u0, N * sizeof(double));
    if (um1) memcpy(uprev, um1, N * sizeof(double));

    const double idz2 = 1.0 / (dz * dz), idx2 = 1.0 / (dx * dx);

    for (int n = 0; n < nt; ++n) {
        /* receiver sampling of u^n */
        if (traces) {
            for (int r = 0; r < nrec; ++r) traces[(size_t)n * nrec + r] = 0.0;
            for (int p = 0; p < nrp; ++p)
                traces[(size_t)n * nrec + rid[p]] += rw[p] * u[IDX(rI[p], rJ[p])];
        }
        if (n == nt - 1) break;

        /* u^{n+1} without the source term */
        for (int I = 0; I < Nz; ++I) {
            for (int J = 0; J < Nx; ++J) {
                double lz = w[0] * u[IDX(I, J)];
                double lx = w[0] * u[IDX(I, J)];
                for (int k = 1; k <= 4; ++k) {
                    double up = (I - k >= 0) ? u[IDX(I - k, J)] : 0.0;
                    double dn = (I + k < Nz) ? u[IDX(I + k, J)] : 0.0;
                    double lf = (J - k >= 0) ? u[IDX(I, J - k)] : 0.0;
                    double rt = (J + k < Nx) ? u[IDX(I, J + k)] : 0.0;
                    lz += w[k] * (up + dn);
                    lx += w[k] * (lf + rt);
                }
                double lap = lz * idz2 + lx * idx2;
                double a = 0.5 * damp[IDX(I, J)] * dt;
                double C = vel[IDX(I, J)] * dt * vel[IDX(I, J)] * dt;
                unext[IDX(I, J)] = (2.0 * u[IDX(I, J)] - (1.0 - a) * uprev[IDX(I, J)] + C * lap) / (1.0 + a);
            }
        }
        /* source term f^n enters the same update, scaled by C/(1+a) */
        if (wavelet) {
            for (int p = 0; p < nsp; ++p) {
                size_t q = IDX(sI[p], sJ[p]);
                double a = 0.5 * damp[q] * dt;
                double C = vel[q] * dt * vel[q] * dt;
                unext[q] += C * sw[p] * wavelet[n] / (dz * dx) / (1.0 + a);
            }
        }
        double *t = uprev; uprev = u; u = unext; unext = t;
    }
    if (ufinal) memcpy(ufinal, u, N * sizeof(double));
    free(u); free(uprev); free(unext);
    return 0;
}
