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

/*
 * Gradient of the l2 misfit with respect to the padded-grid velocity, by the
 * discrete adjoint of the scheme above (TEST INFRASTRUCTURE ONLY).
 *
 *   J = 1/2 sum_{n=0}^{nt-1} sum_r (traces[n][r] - dobs[n][r])^2
 *
 * Dividing the update by C = (v dt)^2 gives the constraint
 *   G^{n+1} = M [(1+a) u^{n+1} - 2 u^n + (1-a) u^{n-1}] - Lap_h u^n - f^n = 0,
 * M = 1/C, whose operator is symmetric (Lap_h is). With psi = -lambda the
 * adjoint runs the same scheme backwards in time with the residual injected
 * at the receiver points:
 *   (1+a) psi^k = 2 psi^{k+1} - (1-a) psi^{k+2} + C (Lap_h psi^{k+1} + r^k),
 *   k = nt-1 .. 1, psi^{nt} = psi^{nt+1} = 0, r^k = P^T (P u^k - dobs^k),
 * and
 *   dJ/dC = sum_{n=0}^{nt-2} psi^{n+1} [(1+a) u^{n+1} - 2 u^n + (1-a) u^{n-1}] / C^2,
 *   dJ/dv = dJ/dC * 2 v dt^2   (u^{-1} = 0).
 * All u^n are kept in memory (small grids only). Returns J in *misfit.
 */
int oracle_gradient_run(
    int Nz, int Nx, double dz, double dx, const double *w, const double *vel, const double *damp,
    double dt, int nt, const double *wavelet,
    int nsp, const int *sI, const int *sJ, const double *sw,
    int nrec, int nrp, const int *rI, const int *rJ, const double *rw, const int *rid,
    const double *dobs,       /* [nt][nrec] observed traces                     */
    double *grad,             /* [Nz][Nx] output: dJ/dv on the padded grid      */
    double *misfit)           /* output: J                                      */
{
    size_t N = (size_t)Nz * (size_t)Nx;
    double *U = calloc(N * (size_t)nt, sizeof(double));        /* u^0 .. u^{nt-1} */
    double *res = calloc((size_t)nt * (size_t)nrec, sizeof(double));
    double *p1 = calloc(N, sizeof(double)), *p2 = calloc(N, sizeof(double)), *p0 = calloc(N, sizeof(double));
    double *gC = calloc(N, sizeof(double));
    if (!U || !res || !p1 || !p2 || !p0 || !gC) {
        free(U); free(res); free(p1); free(p2); free(p0); free(gC);
        return -1;
    }
    const double idz2 = 1.0 / (dz * dz), idx2 = 1.0 / (dx * dx);

    /* forward, keeping every time level */
    for (int n = 0; n + 1 < nt; ++n) {
        const double *u = U + (size_t)n * N;
        const double *um = n > 0 ? U + (size_t)(n - 1) * N : NULL;
        double *un = U + (size_t)(n + 1) * N;
        for (int I = 0; I < Nz; ++I) {
            for (int J = 0; J < Nx; ++J) {
                double lz = w[0] * u[IDX(I, J)], lx = w[0] * u[IDX(I, J)];
                for (int k = 1; k <= 4; ++k) {
                    lz += w[k] * (((I - k >= 0) ? u[IDX(I - k, J)] : 0.0) + ((I + k < Nz) ? u[IDX(I + k, J)] : 0.0));
                    lx += w[k] * (((J - k >= 0) ? u[IDX(I, J - k)] : 0.0) + ((J + k < Nx) ? u[IDX(I, J + k)] : 0.0));
                }
                double a = 0.5 * damp[IDX(I, J)] * dt;
                double C = vel[IDX(I, J)] * dt * vel[IDX(I, J)] * dt;
                double prev = um ? um[IDX(I, J)] : 0.0;
                un[IDX(I, J)] = (2.0 * u[IDX(I, J)] - (1.0 - a) * prev + C * (lz * idz2 + lx * idx2)) / (1.0 + a);
            }
        }
        if (wavelet) {
            for (int p = 0; p < nsp; ++p) {
                size_t q = IDX(sI[p], sJ[p]);
                double a = 0.5 * damp[q] * dt;
                double C = vel[q] * dt * vel[q] * dt;
                un[q] += C * sw[p] * wavelet[n] / (dz * dx) / (1.0 + a);
            }
        }
    }
    /* residuals and misfit */
    double J2 = 0.0;
    for (int n = 0; n < nt; ++n) {
        for (int p = 0; p < nrp; ++p)
            res[(size_t)n * nrec + rid[p]] += rw[p] * U[(size_t)n * N + IDX(rI[p], rJ[p])];
        for (int r = 0; r < nrec; ++r) {
            res[(size_t)n * nrec + r] -= dobs[(size_t)n * nrec + r];
            J2 += res[(size_t)n * nrec + r] * res[(size_t)n * nrec + r];
        }
    }
    *misfit = 0.5 * J2;

    /* adjoint, backwards: p1 = psi^{k+1}, p2 = psi^{k+2}, p0 = psi^k */
    for (int k = nt - 1; k >= 1; --k) {
        for (int I = 0; I < Nz; ++I) {
            for (int J = 0; J < Nx; ++J) {
                double lz = w[0] * p1[IDX(I, J)], lx = w[0] * p1[IDX(I, J)];
                for (int m = 1; m <= 4; ++m) {
                    lz += w[m] * (((I - m >= 0) ? p1[IDX(I - m, J)] : 0.0) + ((I + m < Nz) ? p1[IDX(I + m, J)] : 0.0));
                    lx += w[m] * (((J - m >= 0) ? p1[IDX(I, J - m)] : 0.0) + ((J + m < Nx) ? p1[IDX(I, J + m)] : 0.0));
                }
                double a = 0.5 * damp[IDX(I, J)] * dt;
                double C = vel[IDX(I, J)] * dt * vel[IDX(I, J)] * dt;
                p0[IDX(I, J)] = (2.0 * p1[IDX(I, J)] - (1.0 - a) * p2[IDX(I, J)] + C * (lz * idz2 + lx * idx2)) / (1.0 + a);
            }
        }
        for (int p = 0; p < nrp; ++p) {
            size_t q = IDX(rI[p], rJ[p]);
            double a = 0.5 * damp[q] * dt;
            double C = vel[q] * dt * vel[q] * dt;
            p0[q] += C * rw[p] * res[(size_t)k * nrec + rid[p]] / (1.0 + a);
        }
        /* gradient term of n = k-1: psi^k [(1+a) u^k - 2 u^{k-1} + (1-a) u^{k-2}] */
        const double *uk = U + (size_t)k * N, *uk1 = U + (size_t)(k - 1) * N;
        const double *uk2 = k >= 2 ? U + (size_t)(k - 2) * N : NULL;
        for (size_t q = 0; q < N; ++q) {
            double a = 0.5 * damp[q] * dt;
            double second = (1.0 + a) * uk[q] - 2.0 * uk1[q] + (1.0 - a) * (uk2 ? uk2[q] : 0.0);
            gC[q] += p0[q] * second;
        }
        double *t = p2; p2 = p1; p1 = p0; p0 = t;
    }
    for (size_t q = 0; q < N; ++q) {
        double C = vel[q] * dt * vel[q] * dt;
        grad[q] = gC[q] / (C * C) * 2.0 * vel[q] * dt * dt;
    }
    free(U); free(res); free(p1); free(p2); free(p0); free(gC);
    return 0;
}
