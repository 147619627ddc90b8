// Finite-difference fitness evaluation for gfx950 (MI355X).
//
// Paper: Mojica and Kukreja, arXiv 1905.12795, Testing approach section. The
// fitness of a particle is the l2 misfit between observed traces and traces
// modelled with a 2-D constant-density acoustic finite-difference scheme
// (second order in time, eighth order in space, damping absorbing layer,
// Ricker source, one receiver per surface grid column), summed over shots;
// control-node velocities reach the FD grid by bilinear interpolation.
//
// Layout in HBM (per run = one particle x one shot):
//   two ping-pong pairs of FP32 fields (u_0, v_0) and (u_1, v_1), each field
//   (Nz + 32) rows x S floats, x fastest, the four fields contiguous. A pair
//   holds two consecutive time levels, u^n in u_p and u^{n-1} in v_p. Row s
//   holds padded row I = s - 16 and column c holds padded column J = c - 16;
//   the 16-deep ring around the padded grid and the row tail up to the stride
//   S (a multiple of 64 floats, S >= Nx + 32) stay zero, so the stencil needs
//   no bounds tests. The coefficient field C = (v dt)^2 of a particle uses the
//   same layout and is shared by all of its shots.
// A launch advances every run by T time steps (temporal blocking): it reads
// the pair of parity par and writes the other one.
//
// Kernel shape: one 64-lane wavefront owns a tile of 256 columns (4 adjacent
// columns per lane, 16-byte loads) by bz rows and marches down the rows,
// keeping the 9 rows of each level's z-stencil in registers; x-neighbours
// come from the adjacent lanes by DPP lane shifts. Damping, source injection
// and receiver residuals are fused into the same pass. Tiles are ordered
// particle, z-strip, x-strip, shot (shot fastest) so that the shots of a
// particle read the shared coefficient tile back to back from L2, and block
// indices are remapped so that consecutive tiles run on the same XCD.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace empso {

// ---------------------------------------------------------------------------
// Error state
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

// Eighth-order central weights of the second derivative (Fornberg 1988).
static const double kW[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
// |symbol| at the Nyquist wavenumber: |w0 + 2 sum_k w_k (-1)^k| = 2048/315.
static const double kSymbolMax = 2048.0 / 315.0;

static const int kRing = 16;       // zero ring (rows and columns) around the padded grid
static const int kLanesX = 64;     // lanes per wavefront
static const int kColsPerLane = 4;
static const int kTileX = kLanesX * kColsPerLane;   // columns loaded by one wavefront
static const int kQueue = 10;      // row-queue slots per level (9 stencil rows + 1 prefetch)
static const int kMaxT = 4;        // deepest temporal blocking (4 kMaxT <= kRing)
// The stencil's distance-3 and distance-4 weights are in the exact ratio
// c4 / c3 = -9/128, so c3 (S3 - 4u) + c4 (S4 - 4u) = c3 (S3 - 4 (1 + c4/c3) u) + c4 S4
// with the factor 4 (1 + c4/c3) = 119/32 exact in FP32 (per axis: half of it),
// S_k the sum of the neighbours at distance k: one operation less per point,
// and a constant field still gives an exactly zero Laplacian up to the
// rounding of the coefficients themselves.
static constexpr float kFold3 = 3.71875f;
static constexpr float kFold3Axis = 1.859375f;

}  // namespace empso

using namespace empso;

// ---------------------------------------------------------------------------
// Problem
// ---------------------------------------------------------------------------
struct empso_problem {
    uint64_t uid = 0;          // serial number: never reused, unlike the address
    empso_geometry g;
    int Nz, Nx, S;             // padded sizes, stored row stride (floats)
    int D;                     // node values per particle
    std::vector<int> srcI, srcJ;   // padded indices per shot
    int recI;                  // padded receiver row
    int zlo, zhi;              // stored rows [zlo, zhi) are undamped along z (a_z = 0)
    std::vector<int> reccol;   // padded column of each receiver
    float *d_wav = nullptr;    // [nt]
    float *d_az = nullptr;     // [Nz] a = d dt / 2 along z
    float *d_ax = nullptr;     // [Nx]
    float *d_zoma = nullptr;   // [Nz] 1 - a_z
    float *d_zinv = nullptr;   // [Nz] 1 / (1 + a_z) (the device's reciprocal)
    int *d_recmap = nullptr;   // [Nx] receiver index of a padded column or -1
    int *d_reccol = nullptr;   // [nrec]
    // node-to-grid interpolation tables (regular and layered node grids):
    // row i lies between levels rowa[i] and rowa[i] + 1 at weight rowt[i]
    // (rowa[i] = -1: a water row); on level a, column j lies between nodes
    // cidx[a][j] and cidx[a][j] + 1 (indices into the node vector) at weight cu[a][j]
    int *d_rowa = nullptr;     // [nz]
    float *d_rowt = nullptr;   // [nz]
    int *d_cidx = nullptr;     // [levels][nx]
    float *d_cu = nullptr;     // [levels][nx]
    float c0, cz[4], cx[4], wscale;
};

// Damping factors of the rows: 1 - a_z and the device reciprocal of 1 + a_z,
// the values the stencil kernel's full damped form computes when a_x = 0.
__global__ void k_zfactors(const float *__restrict__ az, int Nz, float *__restrict__ zoma, float *__restrict__ zinv) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < Nz) {
        zoma[I] = 1.0f - az[I];
        zinv[I] = __builtin_amdgcn_rcpf(1.0f + az[I]);
    }
}

extern "C" const char *empso_status_string(int s) {
    switch (s) {
        case EMPSO_OK: return "EMPSO_OK";
        case EMPSO_EINVAL: return "EMPSO_EINVAL";
        case EMPSO_ECFL: return "EMPSO_ECFL";
        case EMPSO_ERANGE: return "EMPSO_ERANGE";
        case EMPSO_EWORKSPACE: return "EMPSO_EWORKSPACE";
        case EMPSO_EHIP: return "EMPSO_EHIP";
        case EMPSO_ENOTSUP: return "EMPSO_ENOTSUP";
        default: return "EMPSO_UNKNOWN";
    }
}

extern "C" const char *empso_last_error(void) { return g_err.c_str(); }

static double stable_dt_raw(double vmax, double dz, double dx) {
    return 2.0 / (vmax * std::sqrt(kSymbolMax * (1.0 / (dz * dz) + 1.0 / (dx * dx))));
}

extern "C" int empso_stable_dt(double vmax, double dz, double dx, double *dt_out) {
    if (!dt_out) EMPSO_FAIL(EMPSO_EINVAL, "dt_out is NULL");
    if (!(vmax > 0) || !(dz > 0) || !(dx > 0) || !std::isfinite(vmax) || !std::isfinite(dz) ||
        !std::isfinite(dx))
        EMPSO_FAIL(EMPSO_EINVAL, "vmax, dz, dx must be positive and finite");
    *dt_out = stable_dt_raw(vmax, dz, dx);
    return EMPSO_OK;
}

// Grid index of a coordinate that must sit on a grid point (tolerance 1e-6 h).
static bool on_grid(double pos, double h, int n, int *idx) {
    double f = pos / h;
    double r = std::nearbyint(f);
    if (std::fabs(f - r) > 1e-6) return false;
    if (r < 0 || r > n - 1) return false;
    *idx = (int)r;
    return true;
}

static void free_problem(empso_problem *p) {
    if (!p) return;
    if (p->d_wav) (void)hipFree(p->d_wav);
    if (p->d_az) (void)hipFree(p->d_az);
    if (p->d_ax) (void)hipFree(p->d_ax);
    if (p->d_zoma) (void)hipFree(p->d_zoma);
    if (p->d_zinv) (void)hipFree(p->d_zinv);
    if (p->d_recmap) (void)hipFree(p->d_recmap);
    if (p->d_reccol) (void)hipFree(p->d_reccol);
    if (p->d_rowa) (void)hipFree(p->d_rowa);
    if (p->d_rowt) (void)hipFree(p->d_rowt);
    if (p->d_cidx) (void)hipFree(p->d_cidx);
    if (p->d_cu) (void)hipFree(p->d_cu);
    delete p;
}

extern "C" int empso_problem_create(const empso_geometry *gp, empso_problem **out) {
    clear_error();
    if (!out) EMPSO_FAIL(EMPSO_EINVAL, "out is NULL");
    *out = nullptr;
    if (!gp) EMPSO_FAIL(EMPSO_EINVAL, "geometry is NULL");
    const empso_geometry &g = *gp;
    if (g.nz < 2 || g.nx < 2 || g.nbl < 0 || g.nt < 1 || g.nshots < 1 || g.nrec < 1)
        EMPSO_FAIL(EMPSO_EINVAL, "sizes must be positive (nz, nx >= 2, nbl >= 0, nt, nshots, nrec >= 1)");
    const bool layered = g.node_z != nullptr;
    int64_t D64 = (int64_t)g.ncz * g.ncx;
    if (!layered) {
        if (g.ncz < 2 || g.ncx < 2) EMPSO_FAIL(EMPSO_EINVAL, "ncz and ncx must be >= 2");
        if (g.ncz > g.nz || g.ncx > g.nx) EMPSO_FAIL(EMPSO_EINVAL, "more control nodes than grid points");
    } else {
        if (g.ncz < 2 || g.ncz > g.nz) EMPSO_FAIL(EMPSO_EINVAL, "a layered grid needs 2 .. nz levels");
        if (!g.level_nodes || !g.node_x) EMPSO_FAIL(EMPSO_EINVAL, "level_nodes / node_x is NULL");
        D64 = 0;
        for (int a = 0; a < g.ncz; ++a) {
            if (!std::isfinite(g.node_z[a]) || (a > 0 && !(g.node_z[a] > g.node_z[a - 1])))
                EMPSO_FAIL(EMPSO_EINVAL, "level depths must be finite and strictly increasing");
            if (g.level_nodes[a] < 2 || g.level_nodes[a] > g.nx)
                EMPSO_FAIL(EMPSO_EINVAL, "level %d: 2 .. nx nodes required", a);
            for (int b = 0; b < g.level_nodes[a]; ++b) {
                const double x = g.node_x[D64 + b];
                if (!std::isfinite(x) || (b > 0 && !(x > g.node_x[D64 + b - 1])))
                    EMPSO_FAIL(EMPSO_EINVAL, "level %d: node x positions must be finite and strictly increasing", a);
            }
            D64 += g.level_nodes[a];
        }
    }
    if (D64 > (1 << 20)) EMPSO_FAIL(EMPSO_ENOTSUP, "too many control nodes");
    if (g.water_rows < 0 || g.water_rows >= g.nz) EMPSO_FAIL(EMPSO_EINVAL, "water_rows must lie in [0, nz)");
    if (g.misfit != EMPSO_MISFIT_L2 && g.misfit != EMPSO_MISFIT_TRACE_NORMALISED)
        EMPSO_FAIL(EMPSO_EINVAL, "misfit must be EMPSO_MISFIT_L2 or EMPSO_MISFIT_TRACE_NORMALISED");
    if (!(g.dz > 0) || !(g.dx > 0) || !(g.dt > 0) || !(g.f0 > 0) || !std::isfinite(g.dz) ||
        !std::isfinite(g.dx) || !std::isfinite(g.dt) || !std::isfinite(g.f0))
        EMPSO_FAIL(EMPSO_EINVAL, "dz, dx, dt, f0 must be positive and finite");
    if (!(g.vmin > 0) || !(g.vmax >= g.vmin) || !std::isfinite(g.vmax))
        EMPSO_FAIL(EMPSO_EINVAL, "need 0 < vmin <= vmax < inf");
    if (!(g.damp_R > 0 && g.damp_R < 1)) EMPSO_FAIL(EMPSO_EINVAL, "damp_R must lie in (0, 1)");
    if (g.water_rows > 0 && !(g.v_water >= g.vmin && g.v_water <= g.vmax))
        EMPSO_FAIL(EMPSO_EINVAL, "v_water must lie in [vmin, vmax]");
    if (!g.src_zx || !g.rec_zx) EMPSO_FAIL(EMPSO_EINVAL, "src_zx / rec_zx is NULL");
    const int64_t Nz64 = (int64_t)g.nz + 2 * (int64_t)g.nbl, Nx64 = (int64_t)g.nx + 2 * (int64_t)g.nbl;
    if (Nz64 > (1 << 20) || Nx64 > (1 << 20) || (Nz64 + 8) * (Nx64 + 72) > (int64_t)1 << 31)
        EMPSO_FAIL(EMPSO_ENOTSUP, "grid too large");
    {
        // the stencil kernel addresses a run's four fields through one buffer
        // resource with 32-bit byte offsets: 4 field bytes must stay below 2^31
        const int64_t S64 = (Nx64 + 2 * kRing + 63) / 64 * 64;
        const int64_t fb64 = ((Nz64 + 2 * kRing) * S64 * (int64_t)sizeof(float) + 255) / 256 * 256;
        if (fb64 >= ((int64_t)1 << 29))
            EMPSO_FAIL(EMPSO_ENOTSUP, "grid too large: a stored field takes %lld bytes (limit 512 MiB)",
                       (long long)fb64);
    }
    if (g.dt > stable_dt_raw(g.vmax, g.dz, g.dx) * (1.0 + 1e-12))
        EMPSO_FAIL(EMPSO_ECFL, "dt = %g exceeds the stability limit %g at vmax = %g", g.dt,
                   stable_dt_raw(g.vmax, g.dz, g.dx), g.vmax);

    static std::atomic<uint64_t> next_uid{1};
    empso_problem *p = new empso_problem();
    p->uid = next_uid.fetch_add(1);
    p->g = g;
    p->g.src_zx = nullptr;
    p->g.rec_zx = nullptr;
    p->g.node_z = nullptr;
    p->g.level_nodes = nullptr;
    p->g.node_x = nullptr;
    p->Nz = (int)Nz64;
    p->Nx = (int)Nx64;
    p->S = (int)align_up((size_t)p->Nx + 2 * kRing, 64);
    p->D = (int)D64;
    for (int s = 0; s < g.nshots; ++s) {
        int i, j;
        if (!on_grid(g.src_zx[2 * s], g.dz, g.nz, &i) || !on_grid(g.src_zx[2 * s + 1], g.dx, g.nx, &j)) {
            free_problem(p);
            EMPSO_FAIL(EMPSO_ENOTSUP, "source %d is not on a grid point of the physical grid", s);
        }
        p->srcI.push_back(i + g.nbl);
        p->srcJ.push_back(j + g.nbl);
    }
    std::vector<int> recmap(p->Nx, -1);
    p->reccol.resize(g.nrec);
    for (int r = 0; r < g.nrec; ++r) {
        int i, j;
        if (!on_grid(g.rec_zx[2 * r], g.dz, g.nz, &i) || !on_grid(g.rec_zx[2 * r + 1], g.dx, g.nx, &j)) {
            free_problem(p);
            EMPSO_FAIL(EMPSO_ENOTSUP, "receiver %d is not on a grid point of the physical grid", r);
        }
        if (r == 0) p->recI = i + g.nbl;
        if (i + g.nbl != p->recI) {
            free_problem(p);
            EMPSO_FAIL(EMPSO_ENOTSUP, "receivers must share one grid row");
        }
        if (recmap[j + g.nbl] >= 0) {
            free_problem(p);
            EMPSO_FAIL(EMPSO_ENOTSUP, "receivers %d and %d share a grid point", recmap[j + g.nbl], r);
        }
        recmap[j + g.nbl] = r;
        p->reccol[r] = j + g.nbl;
    }

    // Ricker wavelet, peak frequency f0, delay 1/f0 (evaluated in FP64, stored FP32)
    std::vector<float> wav(g.nt);
    const double pi = 3.14159265358979323846;
    for (int n = 0; n < g.nt; ++n) {
        double tau = n * g.dt - 1.0 / g.f0;
        double a = pi * pi * g.f0 * g.f0 * tau * tau;
        wav[n] = (float)((1.0 - 2.0 * a) * std::exp(-a));
    }
    // damping a = d dt / 2 with d = d0 (l / nbl)^2 per axis
    std::vector<float> az(p->Nz, 0.f), ax(p->Nx, 0.f);
    if (g.nbl > 0) {
        const double L = std::log(1.0 / g.damp_R);
        const double d0z = 3.0 * g.vmax * L / (2.0 * g.nbl * g.dz);
        const double d0x = 3.0 * g.vmax * L / (2.0 * g.nbl * g.dx);
        for (int I = 0; I < p->Nz; ++I) {
            int l = std::max(0, std::max(g.nbl - I, I - (p->Nz - 1 - g.nbl)));
            double r = (double)l / g.nbl;
            az[I] = (float)(0.5 * g.dt * d0z * r * r);
        }
        for (int J = 0; J < p->Nx; ++J) {
            int l = std::max(0, std::max(g.nbl - J, J - (p->Nx - 1 - g.nbl)));
            double r = (double)l / g.nbl;
            ax[J] = (float)(0.5 * g.dt * d0x * r * r);
        }
    }
    p->zlo = p->zhi = 0;
    for (int I = 0; I < p->Nz; ++I) {
        if (az[I] != 0.f) continue;
        if (p->zhi == 0) p->zlo = I + kRing;
        p->zhi = I + 1 + kRing;
    }
    const double idz2 = 1.0 / (g.dz * g.dz), idx2 = 1.0 / (g.dx * g.dx);
    p->c0 = (float)(kW[0] * (idz2 + idx2));
    for (int k = 0; k < 4; ++k) {
        p->cz[k] = (float)(kW[k + 1] * idz2);
        p->cx[k] = (float)(kW[k + 1] * idx2);
    }
    p->wscale = (float)(1.0 / (g.dz * g.dx));

    // node-to-grid tables, in grid-index units: level a at row position
    // zeta[a], node b of level a at column position xi[a][b]; a regular grid
    // puts its nodes at a (nz-1)/(ncz-1) and b (nx-1)/(ncx-1)
    const int nlev = g.ncz;
    std::vector<double> zeta(nlev);
    std::vector<std::vector<double>> xi(nlev);
    std::vector<int> first(nlev);
    for (int a = 0, k = 0; a < nlev; ++a) {
        const int nb = layered ? g.level_nodes[a] : g.ncx;
        zeta[a] = layered ? g.node_z[a] / g.dz : (double)a * (g.nz - 1) / (g.ncz - 1);
        first[a] = k;
        for (int b = 0; b < nb; ++b)
            xi[a].push_back(layered ? g.node_x[k + b] / g.dx : (double)b * (g.nx - 1) / (g.ncx - 1));
        k += nb;
    }
    std::vector<int> rowa(g.nz), cidx((size_t)nlev * g.nx);
    std::vector<float> rowt(g.nz), cu((size_t)nlev * g.nx);
    for (int i = 0; i < g.nz; ++i) {
        int a = 0;
        double t = 0.0;
        if (i < g.water_rows) {
            a = -1;
        } else if (i <= zeta[0]) {
            a = 0; t = 0.0;
        } else if (i >= zeta[nlev - 1]) {
            a = nlev - 2; t = 1.0;
        } else {
            while (zeta[a + 1] < i) ++a;
            t = (i - zeta[a]) / (zeta[a + 1] - zeta[a]);
        }
        rowa[i] = a;
        rowt[i] = (float)t;
    }
    for (int a = 0; a < nlev; ++a) {
        const std::vector<double> &x = xi[a];
        const int nb = (int)x.size();
        for (int j = 0; j < g.nx; ++j) {
            int b = 0;
            double u = 0.0;
            if (j <= x[0]) {
                b = 0; u = 0.0;
            } else if (j >= x[nb - 1]) {
                b = nb - 2; u = 1.0;
            } else {
                while (x[b + 1] < j) ++b;
                u = (j - x[b]) / (x[b + 1] - x[b]);
            }
            cidx[(size_t)a * g.nx + j] = first[a] + b;
            cu[(size_t)a * g.nx + j] = (float)u;
        }
    }

    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&p->d_rowa, sizeof(int) * g.nz);
    if (e == hipSuccess) e = hipMalloc(&p->d_rowt, sizeof(float) * g.nz);
    if (e == hipSuccess) e = hipMalloc(&p->d_cidx, sizeof(int) * cidx.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_cu, sizeof(float) * cu.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_rowa, rowa.data(), sizeof(int) * g.nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_rowt, rowt.data(), sizeof(float) * g.nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_cidx, cidx.data(), sizeof(int) * cidx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_cu, cu.data(), sizeof(float) * cu.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_wav, sizeof(float) * g.nt);
    if (e == hipSuccess) e = hipMalloc(&p->d_az, sizeof(float) * p->Nz);
    if (e == hipSuccess) e = hipMalloc(&p->d_ax, sizeof(float) * p->Nx);
    if (e == hipSuccess) e = hipMalloc(&p->d_zoma, sizeof(float) * p->Nz);
    if (e == hipSuccess) e = hipMalloc(&p->d_zinv, sizeof(float) * p->Nz);
    if (e == hipSuccess) e = hipMalloc(&p->d_recmap, sizeof(int) * p->Nx);
    if (e == hipSuccess) e = hipMalloc(&p->d_reccol, sizeof(int) * g.nrec);
    if (e == hipSuccess) e = hipMemcpy(p->d_wav, wav.data(), sizeof(float) * g.nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_az, az.data(), sizeof(float) * p->Nz, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_ax, ax.data(), sizeof(float) * p->Nx, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_recmap, recmap.data(), sizeof(int) * p->Nx, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_zfactors<<<(p->Nz + 255) / 256, 256>>>(p->d_az, p->Nz, p->d_zoma, p->d_zinv);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_reccol, p->reccol.data(), sizeof(int) * g.nrec, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_problem(p);
        EMPSO_FAIL(EMPSO_EHIP, "device table upload failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return EMPSO_OK;
}

static void drop_plans_of(uint64_t uid);

extern "C" void empso_problem_destroy(empso_problem *p) {
    if (!p) return;
    drop_plans_of(p->uid);          // cached fitness plans read this problem's tables
    free_problem(p);
}

extern "C" int empso_problem_get_info(const empso_problem *p, empso_problem_info *info) {
    if (!p || !info) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    info->nz = p->g.nz;
    info->nx = p->g.nx;
    info->nbl = p->g.nbl;
    info->nt = p->g.nt;
    info->nshots = p->g.nshots;
    info->nrec = p->g.nrec;
    info->ncz = p->g.ncz;
    info->ncx = p->g.ncx;
    info->Nz = p->Nz;
    info->Nx = p->Nx;
    info->row_stride = p->S;
    info->updates_per_run = (int64_t)p->Nz * p->Nx * (int64_t)(p->g.nt > 0 ? p->g.nt - 1 : 0);
    info->D = p->D;
    return EMPSO_OK;
}

extern "C" int empso_default_tuning(empso_tuning *t) {
    if (!t) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    t->variant = 0;
    t->bz = 160;
    t->tsteps = 4;
    t->prefetch = 1;
    t->use_graph = 1;
    return EMPSO_OK;
}

// ---------------------------------------------------------------------------
// Device-side descriptors
// ---------------------------------------------------------------------------
struct RunDesc {
    float *u[2], *v[2];         // ping-pong pairs (u^n, u^{n-1}) (storage base, ring included)
    const float *C;             // coefficient field of the particle
    const float *obs;           // [nt][nrec] observed traces of this shot (fitness mode)
    float *traces;              // [nt][nrec] output (record mode) or NULL
    double *acc;                // l2: [nrec] running sum of squared residuals;
                                // trace-normalised: [3][nrec] sums of d^2, d o, o^2
    const float *wav, *az, *ax;
    const float *zoma, *zinv;   // [Nz] row factors 1 - a_z, 1 / (1 + a_z)
    const int *recmap, *reccol;
    int Nz, Nx, S, nrec, recS, srcS, srcC, nt;
    int zlo, zhi;               // stored rows [zlo, zhi) have a_z = 0
    int norm;                   // misfit: 0 l2, 1 trace-normalised
    unsigned fbytes;            // bytes of one stored field (u, v or C)
    float c0, cz1, cz2, cz3, cz4, cx1, cx2, cx3, cx4, wscale;
};

// Node-to-grid interpolation tables of a problem (see empso_problem).
struct NodeMap {
    const int *rowa;
    const float *rowt;
    const int *cidx;
    const float *cu;
    int nx;
    float v_water;
};

static NodeMap node_map(const empso_problem *p) {
    return NodeMap{p->d_rowa, p->d_rowt, p->d_cidx, p->d_cu, p->g.nx, (float)p->g.v_water};
}

struct CoefDesc {
    float *C;                   // output coefficient field
    const float *nodes;         // [D] (node mode) or NULL
    const float *vp;            // [nz][nx] (model mode) or NULL
    NodeMap map;
    int nz, nx, nbl, Nz, Nx, S;
    float dt;
};

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Two-grid interpolation at physical grid point (i, j): linear along the two
// levels around row i, then linear between them (bilinear in each cell of a
// regular grid); water rows hold the water velocity.
__device__ __forceinline__ float node_interp(const float *nd, const NodeMap &m, int i, int j) {
    const int a = m.rowa[i];
    if (a < 0) return m.v_water;
    const float t = m.rowt[i];
    const size_t k0 = (size_t)a * m.nx + j, k1 = k0 + m.nx;
    const int b0 = m.cidx[k0], b1 = m.cidx[k1];
    const float u0 = m.cu[k0], u1 = m.cu[k1];
    const float v0 = (1.0f - u0) * nd[b0] + u0 * nd[b0 + 1];
    const float v1 = (1.0f - u1) * nd[b1] + u1 * nd[b1 + 1];
    return (1.0f - t) * v0 + t * v1;
}

__global__ void k_vp_from_nodes(const float *__restrict__ nodes, float *__restrict__ vp, const NodeMap map, int D,
                                int nz, int nx) {
    const int m = blockIdx.y;
    const float *nd = nodes + (size_t)m * D;
    const int64_t npts = (int64_t)nz * nx;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts; k += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(k / nx), j = (int)(k - (int64_t)i * nx);
        vp[(size_t)m * npts + k] = node_interp(nd, map, i, j);
    }
}

// Coefficient field C = (v dt)^2 on the stored layout (zero outside the padded grid).
__global__ void k_coef(const CoefDesc *__restrict__ cds) {
    const CoefDesc cd = cds[blockIdx.y];
    const int rows = cd.Nz + 2 * kRing;
    const int64_t npts = (int64_t)rows * cd.S;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts; k += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(k / cd.S), c = (int)(k - (int64_t)s * cd.S);
        const int I = s - kRing, J = c - kRing;
        float val = 0.0f;
        if (I >= 0 && I < cd.Nz && J >= 0 && J < cd.Nx) {
            const int i = min(max(I - cd.nbl, 0), cd.nz - 1);
            const int j = min(max(J - cd.nbl, 0), cd.nx - 1);
            const float v = cd.nodes ? node_interp(cd.nodes, cd.map, i, j) : cd.vp[(size_t)i * cd.nx + j];
            const float vd = v * cd.dt;
            val = vd * vd;
        }
        cd.C[k] = val;
    }
}

__global__ void k_zero(float4 *__restrict__ p, int64_t n4) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Give each XCD a contiguous range of logical blocks so that neighbouring
// tiles share an L2. The grid is padded to a multiple of 8.
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
    const int per = nblocks >> 3;
    return (b & 7) * per + (b >> 3);
}

// Scalar and vector accesses through explicit address spaces: pointers read
// from descriptors are generic, and generic (flat) accesses count against the
// LDS counter too, so every wait would also wait for all memory in flight.
template <typename T>
__device__ __forceinline__ T gld(const T *p) { return *(const __attribute__((address_space(1))) T *)p; }
template <typename T>
__device__ __forceinline__ void gst(T *p, T v) { *(__attribute__((address_space(1))) T *)p = v; }
// wave-uniform address: scalar load through the constant address space
template <typename T>
__device__ __forceinline__ T sld(const T *p) { return *(const __attribute__((address_space(4))) T *)p; }

typedef float v4f __attribute__((ext_vector_type(4)));

// Raw buffer accesses (MUBUF) with hardware range checking: a load whose byte
// offset lies outside [0, num_records) returns zero and such a store is
// dropped. Offsets are 32-bit, so rows above the field (negative offsets)
// are outside too. kDrop is an offset that is always outside.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
static constexpr int kDrop = (int)0x80000000u;
__device__ __forceinline__ rsrc_t make_rsrc(const float *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float4 bld4(rsrc_t r, int off) {
    const v4f v = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void bst4(rsrc_t r, int off, float4 v) {
    v4f w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, w), r, off, 0, 0);
}

// Trace-normalised misfit: running sums of d^2, d o and o^2 of receiver r
// (the sample products are exact in FP64).
__device__ __forceinline__ void trace_sums(double *acc, int nrec, int r, float d, float o) {
    const double dd = d, oo = o;
    gst(acc + r, gld(acc + r) + dd * dd);
    gst(acc + nrec + r, gld(acc + nrec + r) + dd * oo);
    gst(acc + 2 * nrec + r, gld(acc + 2 * nrec + r) + oo * oo);
}

// Misfit of one trace from its sums: 1/2 |d/sd - o/so|^2 with
// sd = max(|d|, wd), so = max(|o|, wo) (a trace divided by zero stays zero),
// expanded as 1/2 (|d|^2/sd^2 + |o|^2/so^2) - d.o/(sd so). A non-finite
// modelled trace gives +inf.
__device__ __forceinline__ double trace_normalised_misfit(double dd, double dov, double oo, double wd, double wo) {
    if (!(dd < INFINITY) || dov != dov) return INFINITY;
    const double sd = fmax(sqrt(dd), wd), so = fmax(sqrt(oo), wo);
    double m = 0.5 * ((sd > 0.0 ? dd / (sd * sd) : 0.0) + (so > 0.0 ? oo / (so * so) : 0.0));
    if (sd > 0.0 && so > 0.0) m -= dov / (sd * so);
    return fmax(m, 0.0);                            // a sum of squares; the expansion may round below 0
}

// Floor of the trace normalisation of one side (modelled or observed) of a
// shot from its sums of squares ss[nrec]: EMPSO_TRACE_FLOOR times the
// largest trace norm. All threads of the block take part and receive it.
__device__ double trace_floor(const double *ss, int nrec) {
    __shared__ double red[256];
    double m = 0.0;
    for (int r = threadIdx.x; r < nrec; r += blockDim.x) m = fmax(m, ss[r]);
    __syncthreads();
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    const double w = EMPSO_TRACE_FLOOR * sqrt(red[0]);
    __syncthreads();
    return w;
}

// Accumulate (or record) the receiver samples held by one lane: u4 are the
// values of u^n at padded columns J0 .. J0+3 of the receiver row.
__device__ __forceinline__ void sample_receivers(const RunDesc &R, int n, int J0, const float4 ce) {
    const float u4[4] = {ce.x, ce.y, ce.z, ce.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int J = J0 + k;
        if (J >= 0 && J < R.Nx) {
            const int r = gld(R.recmap + J);
            if (r >= 0) {
                const size_t o = (size_t)n * R.nrec + r;
                if (R.traces) {
                    gst(R.traces + o, u4[k]);
                } else if (!R.norm) {
                    const float res = u4[k] - gld(R.obs + o);
                    gst(R.acc + r, gld(R.acc + r) + (double)res * (double)res);
                } else {
                    trace_sums(R.acc, R.nrec, r, u4[k], gld(R.obs + o));
                }
            }
        }
    }
}

// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1): the value of
// lane-1 / lane+1. The lane without a source (0 resp. 63) reads 0 (bound_ctrl).
__device__ __forceinline__ float from_lane_below(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_lane_above(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// T time steps n -> n+T for every tile, all levels in registers.
//
// Fields: each run stores two time levels of u, u^n and u^{n-1}, in two
// ping-pong pairs. The update is the increment form with the increment
// rebuilt from them: dp = u^n - u^{n-1} (a difference of two stored FP32
// values, exact up to one rounding of itself), then
//   d = (C (lap u^n + f^n) + (1 - a) dp) / (1 + a),   u^{n+1} = u^n + d.
// Level t needs u^{n+t-2} at its row, which is the oldest row of level t-1's
// input queue, so no increments are carried between levels.
//
// A wavefront loads 256 columns (4 per lane) and owns the central 256 - 8T of
// them: the level-t result is exact 4t columns in from either edge, so
// neighbouring tiles overlap by 8T columns and recompute them. In z, the
// wavefront owns the rows [s0, s1) its tile names and marches down from 4T
// rows above them, in blocks of 10 steps. In
// each step of the march, level 1 updates row r from u^n rows r-4 .. r+4 (a
// queue of 10 slots with one row requested ahead) and u^{n-1}(r); level t
// updates row r - 4(t-1) from the 9-row queue of level t-1's results and the
// oldest row of level t-1's own queue. Level T writes u^{n+T} and u^{n+T-1}
// for owned rows and columns; every other store gets an out-of-range buffer
// offset and is dropped by the hardware, so the loop body has no branches.
// Rows above or below the stored field read as zero for the same reason.
// Points outside the padded grid need no masking: C is zero there and so are
// the incoming fields, so they stay exactly zero at every level.
// Receiver samples of each level (u^{n+t-1} on the receiver row) are parked
// in LDS and accumulated after the march by the owning lanes; every step
// parks its rows (an extra slot takes those off the receiver row), so the
// step has no branch around the store.
// The damped update d = (C (lap + f) + (1 - a) dp) / (1 + a), a = a_z + a_x,
// is evaluated in the cheapest form that a step's rows and a tile's columns
// allow: with a = 0 as d = C (lap + f) + dp; in a tile holding damped
// columns, on rows with a_z = 0, from per-lane factors 1 - a_x and
// 1 / (1 + a_x); on rows with a_z != 0 in any other tile, from the row
// factors 1 - a_z and 1 / (1 + a_z) (tables built on the device with the
// same reciprocal); otherwise in full. Each form is the full one with a
// zero term, bit for bit, so the results do not depend on the tiling.
//
// Level-keeping mode (KEEP, the misfit gradient's recomputation of a segment): the
// run's fields are a segment's time levels, u^m in field m - b + 1 (b = the
// segment's first step, fields R.fbytes apart from R.u[0]); the launch reads
// u^n and u^{n-1} from fields n - b + 1 and n - b and stores every level's
// owned rows, u^{n+l+1} into field n - b + 2 + l, so all T levels of the
// launch are kept. No receivers are sampled (the descriptor's receiver row
// is one no tile owns).
template <int T, bool ISO, bool KEEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T < 3 ? 3 : 2))) void k_tb(const RunDesc *__restrict__ runs, const int4 *__restrict__ tiles,
                                            int ntiles, int n, int par, int b) {
    constexpr int NS = kQueue;
    constexpr int FILL = 8 * (T - 1);               // march steps before the first owned row
    constexpr int TQ = T > 1 ? T - 1 : 1;
    __shared__ float4 srec[4][T + 1][64];          // slot T: samples of rows off the receiver row
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wv = (int)(threadIdx.x >> 6);
    const int tix = __builtin_amdgcn_readfirstlane(lb * 4 + wv);
    if (tix >= ntiles) return;
    const int lane = threadIdx.x & 63;
    const int4 t = tiles[tix];
    const RunDesc R = runs[t.x];
    const int S = R.S;
    const int bot = R.Nz + kRing;                   // end of the stored rows of the padded grid
    // One buffer resource spans the run's four contiguous fields
    // u0 | u1 | v0 | v1 (pair p = u_p, v_p holds u^n, u^{n-1}); the byte
    // offsets below select the input and output pairs (selects, not
    // R.u[par]: a runtime index would move R to scratch memory). Reads that
    // run past a field land in the next field's zero ring or beyond the range
    // (zero); both only feed rows that are never stored.
    const float *fbase = KEEP ? R.u[0] + (size_t)(n - b) * (R.fbytes >> 2) : R.u[0];
    const rsrc_t F = make_rsrc(fbase, (KEEP ? (unsigned)(T + 2) : 4u) * R.fbytes);
    const int fb = (int)R.fbytes;
    const int uin = (KEEP || par) ? fb : 0, vin = KEEP ? 0 : (par ? 3 * fb : 2 * fb);
    const int uout = par ? 0 : fb, vout = par ? 2 * fb : 3 * fb;
    const rsrc_t Cf = make_rsrc(R.C, R.fbytes);
    const int c = t.z + 4 * lane;                   // stored column of this lane's first element
    // Lanes past the stored row work on its last four columns instead: that
    // tail is zero in every field, the lanes compute zeros there and any
    // store they make writes zeros into the tail, which keeps it zero.
    const int cc = min(c, S - 4);                   // past the row: its zero tail
    const int J0 = c - kRing;
    const bool own = (lane >= T) && (lane < 64 - T);
    const int s0 = t.y;
    const int s1 = min(t.w, bot);                   // the tile's owned stored rows are [s0, s1)
    const int lcol = 4 * cc;                        // byte offset of the lane's columns in a row
    const int rowb = 4 * S;                         // bytes per stored row

    float axk[4], xoma[4], xinv[4], srcm[4];
    bool xdamp = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int J = J0 + k;
        axk[k] = (J >= 0 && J < R.Nx) ? gld(R.ax + J) : 0.0f;
        xoma[k] = 1.0f - axk[k];                        // the factors of a = a_x (rows with a_z = 0)
        xinv[k] = __builtin_amdgcn_rcpf(1.0f + axk[k]);
        xdamp |= axk[k] != 0.0f;
        srcm[k] = (c + k == R.srcC) ? 1.0f : 0.0f;     // this lane holds the source column
    }
    const bool tile_xdamp = __any(xdamp);
    float fsrc[T];
#pragma unroll
    for (int l = 0; l < T; ++l) fsrc[l] = sld(R.wav + min(n + l, R.nt - 1)) * R.wscale;

    const int rs = s0 - 4 * (T - 1);                // level-1 row of the first march step
    float4 q0[NS], qu[TQ][NS], vq, cq[T];
#pragma unroll
    for (int j = 0; j < 9; ++j) q0[j] = bld4(F, uin + (rs - 4 + j) * rowb + lcol);
    vq = bld4(F, vin + rs * rowb + lcol);
#pragma unroll
    for (int l = 0; l < T; ++l) cq[l] = bld4(Cf, (rs - 4 * l) * rowb + lcol);
    // the level queues fill during the first march steps; start them at zero
#pragma unroll
    for (int l = 0; l < TQ; ++l) {
#pragma unroll
        for (int j = 0; j < NS; ++j) qu[l][j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    // One march step: k = (step index) mod 10, known at compile time. Each
    // step takes one form of the update for all its T levels, from the tile
    // (does it hold a damped column) and the step (does any level's row lie
    // in the z layer): undamped, per-lane x factors, row z factors from the
    // tables, or the full damped form.
    auto step = [&](const int k, const int r1, auto mode_tag) __attribute__((always_inline)) {
        // 0: no damping; 1: a = a_x (per-lane factors); 2: a = a_z (row
        // factors from the tables); 3: a = a_z + a_x in full
        constexpr int mode = decltype(mode_tag)::value;
        q0[(k + 9) % NS] = bld4(F, uin + (r1 + 5) * rowb + lcol);
        float4 un = make_float4(0.f, 0.f, 0.f, 0.f), ue = un;
#pragma unroll
        for (int l = 0; l < T; ++l) {
            const float4 *src = (l == 0) ? q0 : qu[l > 0 ? l - 1 : 0];
            const float4 ce = src[(k + 4) % NS];
            const float4 p1 = src[(k + 3) % NS], m1 = src[(k + 5) % NS];
            const float4 p2 = src[(k + 2) % NS], m2 = src[(k + 6) % NS];
            const float4 p3 = src[(k + 1) % NS], m3 = src[(k + 7) % NS];
            const float4 p4 = src[(k + 0) % NS], m4 = src[(k + 8) % NS];
            // u^{n+l-1} at this level's row: loaded for level 1, else the
            // oldest row of the level below's queue
            const float4 pv = (l == 0) ? vq : ((l == 1) ? q0 : qu[l > 1 ? l - 2 : 0])[k % NS];
            const float4 C4 = cq[l];
            const int r = r1 - 4 * l;
            // next step's operands of this level, requested once these are read
            cq[l] = bld4(Cf, (r + 1) * rowb + lcol);
            if (l == 0) vq = bld4(F, vin + (r1 + 1) * rowb + lcol);
            const float v[12] = {from_lane_below(ce.x), from_lane_below(ce.y),
                                 from_lane_below(ce.z), from_lane_below(ce.w),
                                 ce.x, ce.y, ce.z, ce.w,
                                 from_lane_above(ce.x), from_lane_above(ce.y),
                                 from_lane_above(ce.z), from_lane_above(ce.w)};
            const float pz1[4] = {p1.x, p1.y, p1.z, p1.w}, mz1[4] = {m1.x, m1.y, m1.z, m1.w};
            const float pz2[4] = {p2.x, p2.y, p2.z, p2.w}, mz2[4] = {m2.x, m2.y, m2.z, m2.w};
            const float pz3[4] = {p3.x, p3.y, p3.z, p3.w}, mz3[4] = {m3.x, m3.y, m3.z, m3.w};
            const float pz4[4] = {p4.x, p4.y, p4.z, p4.w}, mz4[4] = {m4.x, m4.y, m4.z, m4.w};
            const float pvv[4] = {pv.x, pv.y, pv.z, pv.w};
            const float Cv[4] = {C4.x, C4.y, C4.z, C4.w};
            const int rz = min(max(r - kRing, 0), R.Nz - 1);
            const float azr = (mode == 3) ? sld(R.az + rz) : 0.0f;
            const float zo = (mode == 2) ? sld(R.zoma + rz) : 1.0f;
            const float zi = (mode == 2) ? sld(R.zinv + rz) : 1.0f;
            const float fs = (r == R.srcS) ? fsrc[l] : 0.0f;   // wave-uniform
            float uo[4];
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const float u = v[4 + k2];
                // Laplacian as a sum of small terms, farthest neighbours first:
                // c_k ((u_{+k} + u_{-k}) - 2u) per axis, or with dz = dx
                // c_k (((z pair) + (x pair)) - 4u); the distance-4 pair's
                // share of the centre is folded into the distance-3 term with
                // an exact factor (kFold3). The centre weight is never formed,
                // so no large partial sum cancels (FP32 accuracy over long
                // runs).
                float lap;
                if (ISO) {
                    lap = R.cz4 * ((pz4[k2] + mz4[k2]) + (v[0 + k2] + v[8 + k2]));
                    lap = fmaf(R.cz3, fmaf(-kFold3, u, (pz3[k2] + mz3[k2]) + (v[1 + k2] + v[7 + k2])), lap);
                    lap = fmaf(R.cz2, fmaf(-4.0f, u, (pz2[k2] + mz2[k2]) + (v[2 + k2] + v[6 + k2])), lap);
                    lap = fmaf(R.cz1, fmaf(-4.0f, u, (pz1[k2] + mz1[k2]) + (v[3 + k2] + v[5 + k2])), lap);
                } else {
                    lap = R.cz4 * (pz4[k2] + mz4[k2]);
                    lap = fmaf(R.cz3, fmaf(-kFold3Axis, u, pz3[k2] + mz3[k2]), lap);
                    lap = fmaf(R.cz2, fmaf(-2.0f, u, pz2[k2] + mz2[k2]), lap);
                    lap = fmaf(R.cz1, fmaf(-2.0f, u, pz1[k2] + mz1[k2]), lap);
                    lap = fmaf(R.cx4, v[0 + k2] + v[8 + k2], lap);
                    lap = fmaf(R.cx3, fmaf(-kFold3Axis, u, v[1 + k2] + v[7 + k2]), lap);
                    lap = fmaf(R.cx2, fmaf(-2.0f, u, v[2 + k2] + v[6 + k2]), lap);
                    lap = fmaf(R.cx1, fmaf(-2.0f, u, v[3 + k2] + v[5 + k2]), lap);
                }
                lap = fmaf(srcm[k2], fs, lap);
                const float dp = u - pvv[k2];
                // Every form is the full damped one with some terms known to
                // be zero, and reduces to it bit for bit there (a_z + 0 = a_z,
                // 0 + a_x = a_x, (1-0) dp = dp, rcp(1) = 1), so a point's
                // result does not depend on which form its tile and step take.
                float d;
                if constexpr (mode == 0) {
                    d = fmaf(Cv[k2], lap, dp);
                } else if constexpr (mode == 1) {
                    d = fmaf(Cv[k2], lap, xoma[k2] * dp) * xinv[k2];
                } else if constexpr (mode == 2) {
                    d = fmaf(Cv[k2], lap, zo * dp) * zi;
                } else {
                    const float a = azr + axk[k2];
                    const float inv = __builtin_amdgcn_rcpf(1.0f + a);
                    d = fmaf(Cv[k2], lap, (1.0f - a) * dp) * inv;
                }
                uo[k2] = u + d;
            }
            srec[wv][(r == R.recS) ? l : T][lane] = ce;      // no branch inside the step
            un = make_float4(uo[0], uo[1], uo[2], uo[3]);
            ue = ce;
            if (l < T - 1) qu[l][(k + 8) % NS] = un;
            if constexpr (KEEP) {
                const bool okl = own && (r >= s0) && (r < s1);
                bst4(F, okl ? (2 + l) * fb + r * rowb + lcol : kDrop, un);
            }
        }
        if constexpr (!KEEP) {
            const int rT = r1 - 4 * (T - 1);
            const bool ok = own && (rT >= s0) && (rT < s1);
            const int o = rT * rowb + lcol;
            bst4(F, ok ? uout + o : kDrop, un);            // kDrop: dropped by the range check
            bst4(F, ok ? vout + o : kDrop, ue);
        }
    };

    auto step_any = [&](const int k, const int r1) __attribute__((always_inline)) {
        const bool zrow = r1 - 4 * (T - 1) < R.zlo || r1 >= R.zhi;     // some level's row has a_z != 0
        if (tile_xdamp) {
            if (zrow)
                step(k, r1, std::integral_constant<int, 3>{});
            else
                step(k, r1, std::integral_constant<int, 1>{});
        } else {
            if (zrow)
                step(k, r1, std::integral_constant<int, 2>{});
            else
                step(k, r1, std::integral_constant<int, 0>{});
        }
    };
    // march in blocks of NS steps: the first 8(T-1) steps only fill the
    // level queues and the last block may run past the tile; the stores of
    // those steps are dropped
    const int nit = FILL + (s1 - s0);
    for (int j = 0; j < nit; j += NS) {
#pragma unroll
        for (int kk = 0; kk < NS; ++kk) step_any(kk, rs + j + kk);
    }
    if (R.recS >= s0 && R.recS < s1 && own) {
        // reload the descriptor (the receiver tables need not stay live in
        // scalar registers during the march)
        const RunDesc *Rp = runs + t.x;
        asm volatile("" : "+s"(Rp));
#pragma unroll
        for (int l = 0; l < T; ++l) sample_receivers(*Rp, n + l, J0, srec[wv][l][lane]);
    }
}

// Sample u^n (held in buffer `par`) at the receivers only (the last time sample).
__global__ void k_sample(const RunDesc *__restrict__ runs, int nruns, int n, int par) {
    const int run = blockIdx.y;
    if (run >= nruns) return;
    const RunDesc &R = runs[run];
    const float *u = par ? R.u[1] : R.u[0];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R.nrec; r += gridDim.x * blockDim.x) {
        const float val = u[(size_t)R.recS * R.S + R.reccol[r] + kRing];
        const size_t o = (size_t)n * R.nrec + r;
        if (R.traces) {
            R.traces[o] = val;
        } else if (!R.norm) {
            const float res = val - R.obs[o];
            R.acc[r] += (double)res * (double)res;
        } else {
            trace_sums(R.acc, R.nrec, r, val, R.obs[o]);
        }
    }
}

// fitness[p] = sum over the runs of particle p and their receivers of the
// trace misfit: 1/2 acc (l2) or the trace-normalised misfit of the sums.
// Fixed per-thread order and a fixed tree: the result does not depend on tiling.
__global__ __launch_bounds__(256) void k_fitness(const RunDesc *__restrict__ runs, const int *__restrict__ prun,
                                                 float *__restrict__ fitness) {
    const int p = blockIdx.x;
    double s = 0.0;
    for (int run = prun[p]; run < prun[p + 1]; ++run) {
        const RunDesc &R = runs[run];
        if (R.norm) {
            const double wd = trace_floor(R.acc, R.nrec), wo = trace_floor(R.acc + 2 * R.nrec, R.nrec);
            for (int r = threadIdx.x; r < R.nrec; r += blockDim.x)
                s += trace_normalised_misfit(R.acc[r], R.acc[R.nrec + r], R.acc[2 * R.nrec + r], wd, wo);
        } else {
            for (int r = threadIdx.x; r < R.nrec; r += blockDim.x) s += 0.5 * R.acc[r];
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double f = red[0];
        fitness[p] = (f == f && f < 1e300) ? (float)f : INFINITY;
    }
}

// 1/2 sum (a - b)^2: pass 1 writes one FP64 partial per block, pass 2 sums them.
__global__ __launch_bounds__(256) void k_misfit_partial(const float *__restrict__ a, const float *__restrict__ b,
                                                        int64_t n, double *__restrict__ part) {
    double s = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double r = (double)a[k] - (double)b[k];
        s += r * r;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_misfit_final(const double *__restrict__ part, int nparts, float *out) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += part[k];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(0.5 * red[0]);
}

// ---------------------------------------------------------------------------
// Batch plans: workspace layout, descriptor upload, launch sequence, graphs
// ---------------------------------------------------------------------------
namespace {

struct RunSpec {
    const empso_problem *p;
    int particle;      // index into the coefficient fields
    int shot;
    const float *obs;  // shot's observed traces or NULL
    float *traces;     // record output or NULL
};

static const int kMinBz = 20;      // smallest tile height (sizes the tile tables)
static const int kMaxBz = 1280;    // largest tile height
// tile heights the autotuner tries (each grid is split into balanced strips
// of about that height; tall grids of many runs march best in one or two)
static const int kTuneBz[] = {20, 40, 80, 160, 240, 320, 480, 720, 1040};
static const int kNumTuneBz = (int)(sizeof(kTuneBz) / sizeof(kTuneBz[0]));
static const int kTailBz = 40;     // tile height of the single-step launches that finish the record

static int out_cols(int T) { return kTileX - 8 * T; }

// Height of the z-strips of a grid for tile height bz and depth T: about bz
// rows, balanced over the grid, rounded up so that a strip's march (its
// 8(T-1) queue-fill steps plus its rows) is a whole number of 10-step
// blocks; the last strip takes the rest. Never below ceil(Nz / ceil(Nz/bz)),
// so a grid has at most ceil(Nz/bz) strips.
static int strip_height(const empso_problem *p, int bz, int T) {
    const int nstrips = (p->Nz + bz - 1) / bz;
    const int fill = 8 * (T - 1);
    return ((p->Nz + nstrips - 1) / nstrips + fill + kQueue - 1) / kQueue * kQueue - fill;
}

static int tiles_of(const empso_problem *p, int bz, int T) {
    const int h = strip_height(p, bz, T);
    const int zt = (p->Nz + h - 1) / h;
    const int xt = (p->Nx + out_cols(T) - 1) / out_cols(T);
    return zt * xt;
}

// Upper bound of tiles_of over every valid tuning (bz >= kMinBz, T <= kMaxT):
// sizes the tile tables.
static int tile_capacity(const empso_problem *p) {
    return ((p->Nz + kMinBz - 1) / kMinBz) * ((p->Nx + out_cols(kMaxT) - 1) / out_cols(kMaxT));
}

// stored rows of a field: ring, padded grid, ring
static size_t field_bytes(const empso_problem *p) {
    return align_up((size_t)(p->Nz + 2 * kRing) * p->S * sizeof(float), 256);
}

struct Layout {
    size_t runs_off, tiles_off, tiles1_off, prun_off, coef_off, nodes_off, state_off, acc_off, total;
    size_t hdr_bytes;                      // descriptors + nodes (uploaded each call)
    std::vector<size_t> C_of_particle;     // byte offsets
    std::vector<size_t> field_of_run;      // byte offset of u[0] (u[1], d[0], d[1] follow)
    std::vector<size_t> acc_of_run;
    int ntiles, ntiles1;                   // tiles of the main depth and of single steps
    bool iso;                              // every problem has dz == dx
};

// Workspace layout for the runs (particle-major, shot-minor); independent of
// the tuning except for the tile counts.
static Layout make_layout(const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs, int Dmax,
                          int bz, int T) {
    Layout L;
    const int np = (int)pp.size();
    const int nruns = (int)runs.size();
    int cap = 0;
    L.ntiles = L.ntiles1 = 0;
    L.iso = true;
    for (const RunSpec &r : runs) {
        L.iso = L.iso && (r.p->g.dz == r.p->g.dx);
        cap += tile_capacity(r.p);
        L.ntiles += tiles_of(r.p, bz, T);
        L.ntiles1 += tiles_of(r.p, kTailBz, 1);
    }
    size_t o = 0;
    L.runs_off = o; o = align_up(o + sizeof(RunDesc) * nruns, 256);
    L.tiles_off = o; o = align_up(o + sizeof(int4) * cap, 256);
    L.tiles1_off = o; o = align_up(o + sizeof(int4) * cap, 256);
    L.prun_off = o; o = align_up(o + sizeof(int) * (np + 1), 256);
    L.coef_off = o; o = align_up(o + sizeof(CoefDesc) * np, 256);
    L.nodes_off = o; o = align_up(o + sizeof(float) * (size_t)np * std::max(Dmax, 1), 256);
    L.hdr_bytes = o;
    for (int k = 0; k < np; ++k) {
        L.C_of_particle.push_back(o);
        o += field_bytes(pp[k]);
    }
    L.state_off = o;
    for (int k = 0; k < nruns; ++k) {
        L.field_of_run.push_back(o);
        o += 4 * field_bytes(runs[k].p);
    }
    L.acc_off = o;
    for (int k = 0; k < nruns; ++k) {
        L.acc_of_run.push_back(o);
        const size_t nsums = runs[k].p->g.misfit == EMPSO_MISFIT_TRACE_NORMALISED ? 3 : 1;
        o = align_up(o + sizeof(double) * nsums * runs[k].p->g.nrec, 256);
    }
    L.total = o;
    return L;
}

struct Plan {
    std::vector<const void *> key_ptrs;
    std::vector<int> key_ints;
    std::vector<uint64_t> uids;            // problems the plan was built for
    Layout L;
    std::vector<unsigned char> host_hdr;   // host copy of the descriptor header
    unsigned char *pinned = nullptr;       // pinned staging buffer (hdr_bytes)
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    int progress = -1;                     // time step an evaluation run in blocks has reached (-1: none)
    // release the graph and staging (callers make sure nothing is queued)
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (upload_done) (void)hipEventDestroy(upload_done);
        if (pinned) (void)hipHostFree(pinned);
        exec = nullptr;
        cap_stream = nullptr;
        upload_done = nullptr;
        pinned = nullptr;
        upload_pending = false;
        progress = -1;
    }
    ~Plan() { release(); }
};

static bool same_layout(const Layout &a, const Layout &b) {
    return a.runs_off == b.runs_off && a.tiles_off == b.tiles_off && a.tiles1_off == b.tiles1_off &&
           a.prun_off == b.prun_off && a.coef_off == b.coef_off && a.nodes_off == b.nodes_off &&
           a.state_off == b.state_off && a.acc_off == b.acc_off && a.total == b.total && a.hdr_bytes == b.hdr_bytes &&
           a.C_of_particle == b.C_of_particle && a.field_of_run == b.field_of_run && a.acc_of_run == b.acc_of_run &&
           a.ntiles == b.ntiles && a.ntiles1 == b.ntiles1 && a.iso == b.iso;
}

static std::mutex g_plan_mu;
static std::vector<Plan *> g_plans;   // small LRU
static const size_t kMaxPlans = 8;

static int launch_tb(int T, bool iso, const RunDesc *runs, const int4 *tiles, int ntiles, int n, int par,
                     hipStream_t st) {
    int blocks = (ntiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
#define EMPSO_TB_CASE(TT)                                                                 \
    if (T == TT) {                                                                        \
        if (iso)                                                                          \
            k_tb<TT, true, false><<<blocks, 256, 0, st>>>(runs, tiles, ntiles, n, par, 0);   \
        else                                                                              \
            k_tb<TT, false, false><<<blocks, 256, 0, st>>>(runs, tiles, ntiles, n, par, 0);  \
        return EMPSO_OK;                                                                  \
    }
    EMPSO_TB_CASE(1) EMPSO_TB_CASE(2) EMPSO_TB_CASE(3) EMPSO_TB_CASE(4)
#undef EMPSO_TB_CASE
    return EMPSO_ENOTSUP;
}

// Level-keeping launch (steps n .. n+T-1 of a segment that starts at step b).
static int launch_tb_keep(int T, bool iso, const RunDesc *runs, const int4 *tiles, int ntiles, int n, int b,
                         hipStream_t st) {
    int blocks = (ntiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
#define EMPSO_TB_CASE(TT)                                                                 \
    if (T == TT) {                                                                        \
        if (iso)                                                                          \
            k_tb<TT, true, true><<<blocks, 256, 0, st>>>(runs, tiles, ntiles, n, 0, b);      \
        else                                                                              \
            k_tb<TT, false, true><<<blocks, 256, 0, st>>>(runs, tiles, ntiles, n, 0, b);     \
        return EMPSO_OK;                                                                  \
    }
    EMPSO_TB_CASE(1) EMPSO_TB_CASE(2) EMPSO_TB_CASE(3) EMPSO_TB_CASE(4)
#undef EMPSO_TB_CASE
    return EMPSO_ENOTSUP;
}

// Enqueue the time steps n -> n+1, n0 <= n < n1, of the evaluation on stream
// st: from n0 = 0 first the state is cleared and the coefficients built; the
// time loop runs launches of T steps and single steps for a remainder; at
// n1 = nt - 1 the last sample is taken and (if fitness) the reduction runs.
// n0 is 0 or a multiple of T, so the pair holding the state at n0 is the
// parity of the n0 / T launches before it.
static int enqueue_range(const Plan &pl, unsigned char *ws, int nruns, int np, int nt, const empso_tuning &tu,
                         float *fitness, int n0, int n1, hipStream_t st) {
    const Layout &L = pl.L;
    const RunDesc *runs = reinterpret_cast<const RunDesc *>(ws + L.runs_off);
    const int4 *tiles = reinterpret_cast<const int4 *>(ws + L.tiles_off);
    const int4 *tiles1 = reinterpret_cast<const int4 *>(ws + L.tiles1_off);
    if (n0 == 0) {
        const int64_t n4 = (int64_t)(L.total - L.state_off) / 16;
        k_zero<<<2048, 256, 0, st>>>(reinterpret_cast<float4 *>(ws + L.state_off), n4);
        k_coef<<<dim3(512, np), 256, 0, st>>>(reinterpret_cast<const CoefDesc *>(ws + L.coef_off));
    }
    int n = n0, par = (n0 / tu.tsteps) & 1;
    while (n < n1) {
        int rc;
        if (n + tu.tsteps <= n1) {
            rc = launch_tb(tu.tsteps, L.iso, runs, tiles, L.ntiles, n, par, st);
            n += tu.tsteps;
        } else {
            rc = launch_tb(1, L.iso, runs, tiles1, L.ntiles1, n, par, st);
            n += 1;
        }
        if (rc) return rc;
        par ^= 1;
    }
    if (n1 == nt - 1) {
        k_sample<<<dim3(8, nruns), 256, 0, st>>>(runs, nruns, nt - 1, par);
        if (fitness) k_fitness<<<np, 256, 0, st>>>(runs, reinterpret_cast<const int *>(ws + L.prun_off), fitness);
    }
    return EMPSO_OK;
}

// The whole evaluation on stream st.
static int enqueue_all(const Plan &pl, unsigned char *ws, int nruns, int np, int nt, const empso_tuning &tu,
                       float *fitness, hipStream_t st) {
    return enqueue_range(pl, ws, nruns, np, nt, tu, fitness, 0, nt - 1, st);
}

static void fill_tiles(int4 *td, const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs,
                       int bz, int T) {
    // order: particle, z-strip, x-strip, shot (shot fastest)
    int k = 0;
    size_t r0 = 0;
    const int W = out_cols(T);
    for (size_t q = 0; q < pp.size(); ++q) {
        const empso_problem *p = pp[q];
        size_t r1 = r0;
        while (r1 < runs.size() && runs[r1].particle == (int)q) ++r1;
        const int h = strip_height(p, bz, T);
        const int zt = (p->Nz + h - 1) / h, xt = (p->Nx + W - 1) / W;
        for (int zs = 0; zs < zt; ++zs)
            for (int xs = 0; xs < xt; ++xs)
                for (size_t r = r0; r < r1; ++r)
                    td[k++] = make_int4((int)r, kRing + zs * h, kRing + xs * W - 4 * T,
                                        kRing + std::min((zs + 1) * h, p->Nz));
        r0 = r1;
    }
}

// Build the host copy of the descriptor header.
static void build_header(Plan &pl, unsigned char *ws, const std::vector<const empso_problem *> &pp,
                         const std::vector<RunSpec> &runs, const std::vector<const float *> &vp_of_particle,
                         const double *nodes_h, int ld_nodes, int Dmax, const empso_tuning &tu) {
    const Layout &L = pl.L;
    std::vector<unsigned char> &h = pl.host_hdr;
    h.assign(L.hdr_bytes, 0);
    RunDesc *rd = reinterpret_cast<RunDesc *>(h.data() + L.runs_off);
    int *prun = reinterpret_cast<int *>(h.data() + L.prun_off);
    CoefDesc *cd = reinterpret_cast<CoefDesc *>(h.data() + L.coef_off);
    float *nd = reinterpret_cast<float *>(h.data() + L.nodes_off);
    const int np = (int)pp.size();
    for (int k = 0; k < np; ++k) {
        const empso_problem *p = pp[k];
        CoefDesc &c = cd[k];
        c.C = reinterpret_cast<float *>(ws + L.C_of_particle[k]);
        c.nodes = nullptr;
        c.vp = vp_of_particle.empty() ? nullptr : vp_of_particle[k];
        if (nodes_h) {
            for (int d = 0; d < p->D; ++d) nd[(size_t)k * Dmax + d] = (float)nodes_h[(size_t)k * ld_nodes + d];
            c.nodes = reinterpret_cast<const float *>(ws + L.nodes_off) + (size_t)k * Dmax;
        }
        c.nz = p->g.nz; c.nx = p->g.nx; c.nbl = p->g.nbl;
        c.map = node_map(p);
        c.Nz = p->Nz; c.Nx = p->Nx; c.S = p->S;
        c.dt = (float)p->g.dt;
    }
    int cur = -1;
    for (size_t r = 0; r < runs.size(); ++r) {
        const RunSpec &rs = runs[r];
        const empso_problem *p = rs.p;
        while (cur < rs.particle) prun[++cur] = (int)r;
        RunDesc &d = rd[r];
        float *f = reinterpret_cast<float *>(ws + L.field_of_run[r]);
        const size_t fe = field_bytes(p) / sizeof(float);
        d.u[0] = f; d.u[1] = f + fe; d.v[0] = f + 2 * fe; d.v[1] = f + 3 * fe;
        d.C = reinterpret_cast<const float *>(ws + L.C_of_particle[rs.particle]);
        d.obs = rs.obs; d.traces = rs.traces;
        d.acc = reinterpret_cast<double *>(ws + L.acc_of_run[r]);
        d.wav = p->d_wav; d.az = p->d_az; d.ax = p->d_ax; d.recmap = p->d_recmap; d.reccol = p->d_reccol;
        d.zoma = p->d_zoma; d.zinv = p->d_zinv;
        d.Nz = p->Nz; d.Nx = p->Nx; d.S = p->S; d.nrec = p->g.nrec;
        d.recS = p->recI + kRing;
        d.zlo = p->zlo; d.zhi = p->zhi;
        d.norm = (rs.obs && p->g.misfit == EMPSO_MISFIT_TRACE_NORMALISED) ? 1 : 0;
        d.srcS = p->srcI[rs.shot] + kRing;
        d.srcC = p->srcJ[rs.shot] + kRing;
        d.nt = p->g.nt;
        d.fbytes = (unsigned)field_bytes(p);
        d.c0 = p->c0;
        d.cz1 = p->cz[0]; d.cz2 = p->cz[1]; d.cz3 = p->cz[2]; d.cz4 = p->cz[3];
        d.cx1 = p->cx[0]; d.cx2 = p->cx[1]; d.cx3 = p->cx[2]; d.cx4 = p->cx[3];
        d.wscale = p->wscale;
    }
    while (cur < np) prun[++cur] = (int)runs.size();
    fill_tiles(reinterpret_cast<int4 *>(h.data() + L.tiles_off), pp, runs, tu.bz, tu.tsteps);
    fill_tiles(reinterpret_cast<int4 *>(h.data() + L.tiles1_off), pp, runs, kTailBz, 1);
}

// Upload the plan's descriptor header through its pinned staging buffer.
static int upload_header(Plan *pl, unsigned char *ws, hipStream_t st) {
    if (!pl->pinned) {
        EMPSO_HIP(hipHostMalloc(reinterpret_cast<void **>(&pl->pinned), pl->L.hdr_bytes, hipHostMallocDefault));
        EMPSO_HIP(hipEventCreateWithFlags(&pl->upload_done, hipEventDisableTiming));
    }
    if (pl->upload_pending) EMPSO_HIP(hipEventSynchronize(pl->upload_done));
    std::memcpy(pl->pinned, pl->host_hdr.data(), pl->L.hdr_bytes);
    EMPSO_HIP(hipMemcpyAsync(ws, pl->pinned, pl->L.hdr_bytes, hipMemcpyHostToDevice, st));
    EMPSO_HIP(hipEventRecord(pl->upload_done, st));
    pl->upload_pending = true;
    return EMPSO_OK;
}

static int run_plan(Plan *pl, unsigned char *ws, int nruns, int np, int nt, const empso_tuning &tu, float *fitness,
                    hipStream_t st) {
    const int urc = upload_header(pl, ws, st);
    if (urc) return urc;
    pl->progress = -1;

    if (!tu.use_graph) {
        int rc = enqueue_all(*pl, ws, nruns, np, nt, tu, fitness, st);
        if (rc) EMPSO_FAIL(rc, "launch failed");
        EMPSO_HIP(hipGetLastError());
        return EMPSO_OK;
    }
    if (!pl->exec) {
        if (!pl->cap_stream) EMPSO_HIP(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        EMPSO_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_all(*pl, ws, nruns, np, nt, tu, fitness, pl->cap_stream);
        hipError_t e = hipStreamEndCapture(pl->cap_stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            EMPSO_FAIL(rc, "launch failed during capture");
        }
        if (e != hipSuccess) EMPSO_FAIL(EMPSO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            pl->exec = nullptr;
            EMPSO_FAIL(EMPSO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    EMPSO_HIP(hipGraphLaunch(pl->exec, st));
    return EMPSO_OK;
}

// Any call that writes a workspace ends every evaluation in blocks on it.
// The caller holds g_plan_mu.
static void forget_progress(const void *ws) {
    for (Plan *p : g_plans)
        if (!p->key_ptrs.empty() && p->key_ptrs[0] == ws) p->progress = -1;
}

static Plan *find_or_make_plan(const std::vector<const void *> &kp, const std::vector<int> &ki, bool *fresh) {
    for (size_t i = 0; i < g_plans.size(); ++i) {
        Plan *p = g_plans[i];
        if (p->key_ptrs == kp && p->key_ints == ki) {
            g_plans.erase(g_plans.begin() + i);
            g_plans.push_back(p);
            *fresh = false;
            return p;
        }
    }
    if (g_plans.size() >= kMaxPlans) {
        Plan *old = g_plans.front();
        // make sure nothing of the evicted plan is still queued before freeing
        (void)hipDeviceSynchronize();
        delete old;
        g_plans.erase(g_plans.begin());
    }
    Plan *p = new Plan();
    p->key_ptrs = kp;
    p->key_ints = ki;
    g_plans.push_back(p);
    *fresh = true;
    return p;
}

}  // namespace

// Forward-modelling tunings chosen by timing, per (problem serial, shot count).
static std::map<std::pair<uint64_t, int>, empso_tuning> g_fwd_tuning;

static void drop_plans_of(uint64_t uid) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_fwd_tuning.begin(); it != g_fwd_tuning.end();)
        it = (it->first.first == uid) ? g_fwd_tuning.erase(it) : std::next(it);
    bool synced = false;
    for (size_t i = 0; i < g_plans.size();) {
        Plan *pl = g_plans[i];
        if (std::find(pl->uids.begin(), pl->uids.end(), uid) != pl->uids.end()) {
            if (!synced) {
                (void)hipDeviceSynchronize();     // nothing of the plan may still be queued
                synced = true;
            }
            delete pl;
            g_plans.erase(g_plans.begin() + i);
        } else {
            ++i;
        }
    }
}

namespace {

static bool valid_tuning(const empso_tuning &t) {
    return t.bz >= 20 && t.bz <= kMaxBz && t.bz % 20 == 0 && t.tsteps >= 1 && t.tsteps <= kMaxT && t.prefetch == 1 &&
           (t.use_graph == 0 || t.use_graph == 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Public entry points
// ---------------------------------------------------------------------------
extern "C" int empso_vp_from_nodes(const empso_problem *p, int32_t nmodels, const float *nodes_d, float *vp_d,
                                   empso_stream stream) {
    clear_error();
    if (!p || !nodes_d || !vp_d) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nmodels < 1 || nmodels > 65535) EMPSO_FAIL(EMPSO_EINVAL, "nmodels must be in [1, 65535]");
    const int64_t npts = (int64_t)p->g.nz * p->g.nx;
    const int bx = (int)std::min<int64_t>(1024, (npts + 255) / 256);
    k_vp_from_nodes<<<dim3(bx, nmodels), 256, 0, (hipStream_t)stream>>>(nodes_d, vp_d, node_map(p), p->D, p->g.nz,
                                                                         p->g.nx);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

extern "C" size_t empso_misfit_workspace_bytes(int64_t n) {
    (void)n;
    return 1024 * sizeof(double);
}

extern "C" int empso_misfit(const float *a_d, const float *b_d, int64_t n, float *out_d, void *ws, size_t ws_bytes,
                            empso_stream stream) {
    clear_error();
    if (!out_d || !ws || (n > 0 && (!a_d || !b_d))) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (n < 0) EMPSO_FAIL(EMPSO_EINVAL, "n must be >= 0");
    if (ws_bytes < empso_misfit_workspace_bytes(n)) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const int nb = 1024;
    k_misfit_partial<<<nb, 256, 0, st>>>(a_d, b_d, n, reinterpret_cast<double *>(ws));
    k_misfit_final<<<1, 256, 0, st>>>(reinterpret_cast<const double *>(ws), nb, out_d);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

// Sums over time (in order, as the fitness kernels accumulate them) of each
// recorded trace (shot blockIdx.y, receiver r) into sums[shot][k][nrec]:
// l2: k = 0 the squared residuals; trace-normalised: k = 0, 1, 2 the sums of
// d^2, d o and o^2.
__global__ __launch_bounds__(256) void k_trace_sums(const float *__restrict__ d, const float *__restrict__ o,
                                                    int nt, int nrec, int norm, double *__restrict__ sums) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const size_t base = (size_t)blockIdx.y * nt * nrec + r;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int n = 0; n < nt; ++n) {
        const float dv = d[base + (size_t)n * nrec], ov = o[base + (size_t)n * nrec];
        if (norm) {
            a += (double)dv * dv;
            b += (double)dv * ov;
            c += (double)ov * ov;
        } else {
            const float res = dv - ov;
            a += (double)res * (double)res;
        }
    }
    double *q = sums + (size_t)blockIdx.y * 3 * nrec + r;
    q[0] = a;
    q[nrec] = b;
    q[2 * nrec] = c;
}

// Misfit of each trace of shot blockIdx.x from its sums into per[shot][nrec].
__global__ __launch_bounds__(256) void k_trace_misfit(const double *__restrict__ sums, int nrec, int norm,
                                                      double *__restrict__ per) {
    const double *q = sums + (size_t)blockIdx.x * 3 * nrec;
    const double wd = norm ? trace_floor(q, nrec) : 0.0, wo = norm ? trace_floor(q + 2 * nrec, nrec) : 0.0;
    for (int r = threadIdx.x; r < nrec; r += blockDim.x)
        per[(size_t)blockIdx.x * nrec + r] =
            norm ? trace_normalised_misfit(q[r], q[nrec + r], q[2 * nrec + r], wd, wo) : 0.5 * q[r];
}

// out = sum of n values in a fixed order; not finite -> +inf.
__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ v, int64_t n, float *out) {
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) s += v[k];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (red[0] == red[0] && red[0] < 1e300) ? (float)red[0] : INFINITY;
}

extern "C" size_t empso_traces_misfit_workspace_bytes(const empso_problem *p, int32_t nsh) {
    if (!p || nsh < 0) return 0;
    return align_up(sizeof(double) * 4 * (size_t)std::max(nsh, 1) * p->g.nrec, 256);
}

// Enqueue the traces misfit with its scratch (4 nsh nrec doubles) at ws.
static int enqueue_traces_misfit(const empso_problem *p, const float *traces_d, const float *obs_d, int32_t nsh,
                                 float *out_d, double *ws, hipStream_t st) {
    const int nrec = p->g.nrec;
    double *sums = ws;                                             // [nsh][3][nrec]
    double *per = sums + (size_t)3 * nsh * nrec;                   // [nsh][nrec]
    const int norm = p->g.misfit == EMPSO_MISFIT_TRACE_NORMALISED ? 1 : 0;
    if (nsh > 0) {
        k_trace_sums<<<dim3((nrec + 255) / 256, nsh), 256, 0, st>>>(traces_d, obs_d, p->g.nt, nrec, norm, sums);
        k_trace_misfit<<<nsh, 256, 0, st>>>(sums, nrec, norm, per);
    }
    k_sum_final<<<1, 256, 0, st>>>(per, (int64_t)nsh * nrec, out_d);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

extern "C" int empso_traces_misfit(const empso_problem *p, const float *traces_d, const float *obs_d, int32_t nsh,
                                   float *out_d, void *ws, size_t ws_bytes, empso_stream stream) {
    clear_error();
    if (!p || !out_d || !ws || (nsh > 0 && (!traces_d || !obs_d))) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nsh < 0) EMPSO_FAIL(EMPSO_EINVAL, "nsh must be >= 0");
    if (ws_bytes < empso_traces_misfit_workspace_bytes(p, nsh)) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    return enqueue_traces_misfit(p, traces_d, obs_d, nsh, out_d, reinterpret_cast<double *>(ws),
                                 (hipStream_t)stream);
}

// Scratch of empso_traces_misfit_noalloc: one array per GPU for the life of
// the process. In host code `scratch` names a host-side stand-in; kernels get
// the device address that hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchDoubles = (size_t)4 * EMPSO_NOALLOC_MAX_TRACES;
static __device__ __align__(256) double scratch[kScratchDoubles];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];      // device address of scratch per device (NULL: not looked up)

// A second stream per device for work that overlaps the caller's stream
// (non-blocking, default priority), created on first use and kept until the
// process ends. Calls that use it on one device share it, so their
// overlapped parts run one after another; events order it against the
// caller's stream.
static std::mutex g_side_mu;
static hipStream_t g_side[kMaxDevices];
static int side_stream(hipStream_t *out) {
    int dev = 0;
    EMPSO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) EMPSO_FAIL(EMPSO_ENOTSUP, "device %d beyond the library's table", dev);
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[dev]) EMPSO_HIP(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return EMPSO_OK;
}

static int scratch_of_current_device(double **out) {
    int dev = 0;
    EMPSO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) EMPSO_FAIL(EMPSO_ENOTSUP, "device %d beyond the %d this call supports", dev,
                                                  kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            EMPSO_FAIL(EMPSO_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return EMPSO_OK;
}

extern "C" int empso_traces_misfit_noalloc(const empso_problem *p, const float *traces_d, const float *obs_d,
                                           int32_t nsh, float *out_d, empso_stream stream) {
    clear_error();
    if (!p || !out_d || (nsh > 0 && (!traces_d || !obs_d))) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nsh < 0) EMPSO_FAIL(EMPSO_EINVAL, "nsh must be >= 0");
    if ((int64_t)nsh * p->g.nrec > EMPSO_NOALLOC_MAX_TRACES)
        EMPSO_FAIL(EMPSO_ENOTSUP, "nsh * nrec = %lld traces exceed the fixed scratch of %d traces",
                   (long long)nsh * p->g.nrec, (int)EMPSO_NOALLOC_MAX_TRACES);
    double *ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    return enqueue_traces_misfit(p, traces_d, obs_d, nsh, out_d, ws, (hipStream_t)stream);
}

static void forward_specs(const empso_problem *p, int32_t shot0, int32_t nsh, float *traces_d,
                          std::vector<const empso_problem *> &pp, std::vector<RunSpec> &runs) {
    pp.assign(1, p);
    runs.clear();
    for (int s = 0; s < nsh; ++s)
        runs.push_back(RunSpec{p, 0, shot0 + s, nullptr, traces_d + (size_t)s * p->g.nt * p->g.nrec});
}

extern "C" size_t empso_forward_workspace_bytes(const empso_problem *p, int32_t nsh) {
    if (!p || nsh < 1) return 0;
    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    forward_specs(p, 0, nsh, nullptr, pp, runs);
    return make_layout(pp, runs, p->D, kMinBz, kMaxT).total;
}

static int forward_autotune(const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs,
                            const std::vector<const float *> &vps, unsigned char *w, hipStream_t st,
                            empso_tuning *best);

extern "C" int empso_forward_shots(const empso_problem *p, const float *vp_d, int32_t shot0, int32_t nsh,
                                   float *traces_d, void *ws, size_t ws_bytes, const empso_tuning *tuning,
                                   empso_stream stream) {
    clear_error();
    if (!p) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nsh < 0 || shot0 < 0 || shot0 + nsh > p->g.nshots) EMPSO_FAIL(EMPSO_EINVAL, "shot range out of bounds");
    if (nsh == 0) return EMPSO_OK;              // empty shot range: nothing to model or enqueue
    if (!vp_d || !traces_d || !ws) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256) EMPSO_FAIL(EMPSO_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < empso_forward_workspace_bytes(p, nsh)) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    // range check of the model on the host (guarantees the CFL condition)
    std::vector<float> vh((size_t)p->g.nz * p->g.nx);
    EMPSO_HIP(hipMemcpyAsync(vh.data(), vp_d, vh.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    EMPSO_HIP(hipStreamSynchronize(st));
    for (size_t k = 0; k < vh.size(); ++k)
        if (!(vh[k] >= (float)p->g.vmin && vh[k] <= (float)p->g.vmax) || !std::isfinite(vh[k]))
            EMPSO_FAIL(EMPSO_ERANGE, "vp[%zu] = %g outside [%g, %g]", k, (double)vh[k], p->g.vmin, p->g.vmax);

    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    forward_specs(p, shot0, nsh, traces_d, pp, runs);
    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    std::vector<const float *> vps(1, vp_d);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    empso_tuning tu;
    if (tuning) {
        tu = *tuning;
    } else {
        // timed once per problem and shot count: the best tiling of a few
        // runs differs from that of a large fitness batch
        const auto key = std::make_pair(p->uid, (int)nsh);
        const auto it = g_fwd_tuning.find(key);
        if (it != g_fwd_tuning.end()) {
            tu = it->second;
        } else {
            const int rc = forward_autotune(pp, runs, vps, w, st, &tu);
            if (rc) return rc;
            g_fwd_tuning[key] = tu;
        }
    }
    tu.use_graph = 0;
    if (!valid_tuning(tu)) EMPSO_FAIL(EMPSO_ENOTSUP, "unsupported tuning");
    forget_progress(w);
    Plan pl;
    pl.L = make_layout(pp, runs, p->D, tu.bz, tu.tsteps);
    build_header(pl, w, pp, runs, vps, nullptr, 0, p->D, tu);
    int rc = run_plan(&pl, w, (int)runs.size(), 1, p->g.nt, tu, nullptr, st);
    if (rc) return rc;
    // the staging buffer is freed with the local plan: wait for the upload
    EMPSO_HIP(hipEventSynchronize(pl.upload_done));
    return EMPSO_OK;
}

static int batch_specs(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                       const int32_t *pop, int32_t np, std::vector<const empso_problem *> &pp,
                       std::vector<RunSpec> &runs, int *Dmax) {
    pp.clear();
    runs.clear();
    *Dmax = 0;
    for (int k = 0; k < np; ++k) {
        const int q = pop[k];
        if (q < 0 || q >= nprob) EMPSO_FAIL(EMPSO_EINVAL, "prob_of_particle[%d] = %d out of range", k, q);
        const empso_problem *p = probs[q];
        if (!p) EMPSO_FAIL(EMPSO_EINVAL, "probs[%d] is NULL", q);
        pp.push_back(p);
        *Dmax = std::max(*Dmax, p->D);
        for (int s = 0; s < p->g.nshots; ++s)
            runs.push_back(RunSpec{p, k, s, obs_d ? obs_d[q] + (size_t)s * p->g.nt * p->g.nrec : nullptr, nullptr});
    }
    return EMPSO_OK;
}

extern "C" size_t empso_fitness_workspace_bytes(const empso_problem *const *probs, int32_t nprob,
                                                const int32_t *pop, int32_t np) {
    if (!probs || !pop || nprob < 1 || np < 1) return 0;
    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    int Dmax;
    if (batch_specs(probs, nprob, nullptr, pop, np, pp, runs, &Dmax)) return 0;
    return make_layout(pp, runs, Dmax, kMinBz, kMaxT).total;
}

// Validation and plan lookup shared by empso_fitness_batch and
// empso_fitness_batch_steps. check_nodes: range-check nodes_h on the host.
// On success *plp is the batch's plan (the caller holds g_plan_mu) and
// *fresh tells whether it was built anew.
struct BatchCall {
    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    int Dmax = 0;
    empso_tuning tu;
};

static int batch_call(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d, const int32_t *pop,
                      int32_t np, const double *nodes_h, int32_t ld_nodes, const float *fitness_d, void *ws,
                      size_t ws_bytes, const empso_tuning *tuning, bool check_nodes, BatchCall &bc,
                      std::vector<const void *> &kp, std::vector<int> &ki, std::vector<uint64_t> &uids) {
    if (!probs || !obs_d || !pop || (check_nodes && !nodes_h) || !fitness_d || !ws)
        EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nprob < 1 || np < 1) EMPSO_FAIL(EMPSO_EINVAL, "nprob >= 1 and np >= 0 required");
    if (reinterpret_cast<uintptr_t>(ws) % 256) EMPSO_FAIL(EMPSO_EINVAL, "workspace must be 256-byte aligned");
    for (int q = 0; q < nprob; ++q) {
        if (!probs[q]) EMPSO_FAIL(EMPSO_EINVAL, "probs[%d] is NULL", q);
        if (!obs_d[q]) EMPSO_FAIL(EMPSO_EINVAL, "obs_d[%d] is NULL", q);
        if (probs[q]->g.nt != probs[0]->g.nt) EMPSO_FAIL(EMPSO_ENOTSUP, "all problems of a batch must share nt");
    }
    if (tuning) bc.tu = *tuning; else empso_default_tuning(&bc.tu);
    if (!valid_tuning(bc.tu)) EMPSO_FAIL(EMPSO_ENOTSUP, "unsupported tuning");
    int rc = batch_specs(probs, nprob, obs_d, pop, np, bc.pp, bc.runs, &bc.Dmax);
    if (rc) return rc;
    if (check_nodes) {
        if (ld_nodes < bc.Dmax) EMPSO_FAIL(EMPSO_EINVAL, "ld_nodes = %d < %d", ld_nodes, bc.Dmax);
        // range check on the host in FP64: bilinear interpolation is a convex
        // combination, so every grid velocity then lies in [vmin, vmax] and the
        // stability condition checked at problem creation holds everywhere.
        for (int k = 0; k < np; ++k) {
            const empso_problem *p = bc.pp[k];
            for (int d = 0; d < p->D; ++d) {
                const double v = nodes_h[(size_t)k * ld_nodes + d];
                if (!(v >= p->g.vmin && v <= p->g.vmax))
                    EMPSO_FAIL(EMPSO_ERANGE, "node %d of particle %d = %g outside [%g, %g]", d, k, v, p->g.vmin,
                               p->g.vmax);
            }
        }
    }
    const size_t need = make_layout(bc.pp, bc.runs, bc.Dmax, kMinBz, kMaxT).total;
    if (ws_bytes < need) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);

    // plan key: buffers, problems by serial number (a destroyed problem's
    // address can come back for a new one), batch composition and tuning
    kp.push_back(ws);
    kp.push_back(fitness_d);
    for (int q = 0; q < nprob; ++q) {
        uids.push_back(probs[q]->uid);
        ki.push_back((int)(probs[q]->uid & 0x7fffffff));
        ki.push_back((int)(probs[q]->uid >> 31));
    }
    ki.push_back(np);
    ki.push_back(bc.tu.bz);
    ki.push_back(bc.tu.tsteps);
    ki.push_back(bc.tu.prefetch);
    for (int k = 0; k < np; ++k) ki.push_back(pop[k]);
    return EMPSO_OK;
}

// The batch's plan, rebuilt if its layout changed. The caller holds g_plan_mu.
static Plan *batch_plan(BatchCall &bc, const std::vector<const void *> &kp, const std::vector<int> &ki,
                        const std::vector<uint64_t> &uids, bool *fresh) {
    Plan *pl = find_or_make_plan(kp, ki, fresh);
    Layout Lnow = make_layout(bc.pp, bc.runs, bc.Dmax, bc.tu.bz, bc.tu.tsteps);
    if (!*fresh && !same_layout(pl->L, Lnow)) {
        // never replay a plan built for another layout: rebuild it
        (void)hipDeviceSynchronize();
        pl->release();
        *fresh = true;
    }
    if (*fresh) {
        pl->L = std::move(Lnow);
        pl->uids = uids;
    }
    return pl;
}

extern "C" int empso_fitness_batch(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                                   const int32_t *pop, int32_t np, const double *nodes_h, int32_t ld_nodes,
                                   float *fitness_d, void *ws, size_t ws_bytes, const empso_tuning *tuning,
                                   empso_stream stream) {
    clear_error();
    if (np == 0) return EMPSO_OK;               // empty batch: nothing to evaluate or enqueue
    BatchCall bc;
    std::vector<const void *> kp;
    std::vector<int> ki;
    std::vector<uint64_t> uids;
    int rc = batch_call(probs, nprob, obs_d, pop, np, nodes_h, ld_nodes, fitness_d, ws, ws_bytes, tuning, true, bc,
                        kp, ki, uids);
    if (rc) return rc;
    ki.push_back(bc.tu.use_graph);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    bool fresh;
    Plan *pl = batch_plan(bc, kp, ki, uids, &fresh);
    forget_progress(ws);
    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    build_header(*pl, w, bc.pp, bc.runs, std::vector<const float *>(), nodes_h, ld_nodes, bc.Dmax, bc.tu);
    return run_plan(pl, w, (int)bc.runs.size(), np, bc.pp[0]->g.nt, bc.tu, fitness_d, (hipStream_t)stream);
}

extern "C" int empso_fitness_batch_steps(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                                         const int32_t *pop, int32_t np, const double *nodes_h, int32_t ld_nodes,
                                         float *fitness_d, int32_t n_begin, int32_t n_end, void *ws, size_t ws_bytes,
                                         const empso_tuning *tuning, empso_stream stream) {
    clear_error();
    if (np == 0) return EMPSO_OK;               // empty batch: nothing to evaluate or enqueue
    BatchCall bc;
    std::vector<const void *> kp;
    std::vector<int> ki;
    std::vector<uint64_t> uids;
    int rc = batch_call(probs, nprob, obs_d, pop, np, nodes_h, ld_nodes, fitness_d, ws, ws_bytes, tuning,
                        n_begin == 0, bc, kp, ki, uids);
    if (rc) return rc;
    const int nt = bc.pp[0]->g.nt, T = bc.tu.tsteps;
    if (n_begin < 0 || n_end < n_begin || n_end > nt - 1)
        EMPSO_FAIL(EMPSO_EINVAL, "need 0 <= n_begin <= n_end <= nt - 1 = %d (got %d, %d)", nt - 1, n_begin, n_end);
    if (n_begin % T != 0 || (n_end != nt - 1 && n_end % T != 0))
        EMPSO_FAIL(EMPSO_EINVAL, "n_begin must be a multiple of tsteps = %d, n_end one too or nt - 1", T);
    ki.push_back(2);                            // block calls never share a plan with graph replay
    std::lock_guard<std::mutex> lk(g_plan_mu);
    bool fresh;
    Plan *pl = batch_plan(bc, kp, ki, uids, &fresh);
    if (n_begin > 0 && (fresh || pl->progress != n_begin))
        EMPSO_FAIL(EMPSO_EINVAL, "no evaluation of this batch on this workspace stands at step %d", n_begin);
    const int at = pl->progress;
    forget_progress(ws);
    pl->progress = at;
    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    hipStream_t st = (hipStream_t)stream;
    if (n_begin == 0) {
        build_header(*pl, w, bc.pp, bc.runs, std::vector<const float *>(), nodes_h, ld_nodes, bc.Dmax, bc.tu);
        rc = upload_header(pl, w, st);
        if (rc) return rc;
    }
    pl->progress = -1;
    rc = enqueue_range(*pl, w, (int)bc.runs.size(), np, nt, bc.tu, fitness_d, n_begin, n_end, st);
    if (rc) EMPSO_FAIL(rc, "launch failed");
    EMPSO_HIP(hipGetLastError());
    pl->progress = n_end < nt - 1 ? n_end : -1;
    return EMPSO_OK;
}

// ---------------------------------------------------------------------------
// Timing of one tuning and the autotuner built on it. Every valid tuning gives
// identical results, so the choice only affects speed.
// ---------------------------------------------------------------------------
static int batch_prepare(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                         const int32_t *pop, int32_t np, const double *nodes_h, int32_t ld_nodes, void *ws,
                         size_t ws_bytes, std::vector<const empso_problem *> &pp, std::vector<RunSpec> &runs,
                         int *Dmax) {
    if (!probs || !obs_d || !pop || !nodes_h || !ws) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (nprob < 1 || np < 1) EMPSO_FAIL(EMPSO_EINVAL, "nprob and np must be >= 1");
    if (reinterpret_cast<uintptr_t>(ws) % 256) EMPSO_FAIL(EMPSO_EINVAL, "workspace must be 256-byte aligned");
    for (int q = 0; q < nprob; ++q) {
        if (!probs[q] || !obs_d[q]) EMPSO_FAIL(EMPSO_EINVAL, "probs[%d] or obs_d[%d] is NULL", q, q);
        if (probs[q]->g.nt != probs[0]->g.nt) EMPSO_FAIL(EMPSO_ENOTSUP, "all problems of a batch must share nt");
    }
    int rc = batch_specs(probs, nprob, obs_d, pop, np, pp, runs, Dmax);
    if (rc) return rc;
    if (ld_nodes < *Dmax) EMPSO_FAIL(EMPSO_EINVAL, "ld_nodes = %d < %d", ld_nodes, *Dmax);
    for (int k = 0; k < np; ++k)
        for (int d = 0; d < pp[k]->D; ++d) {
            const double v = nodes_h[(size_t)k * ld_nodes + d];
            if (!(v >= pp[k]->g.vmin && v <= pp[k]->g.vmax))
                EMPSO_FAIL(EMPSO_ERANGE, "node %d of particle %d = %g outside [%g, %g]", d, k, v, pp[k]->g.vmin,
                           pp[k]->g.vmax);
        }
    if (ws_bytes < make_layout(pp, runs, *Dmax, kMinBz, kMaxT).total)
        EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    return EMPSO_OK;
}

// Set up the batch for tuning tu (header, zero state, coefficients), run
// `warm` untimed and `reps` timed launches of depth tu.tsteps from time 0.
// The coefficient fields come from the particles' node values (nodes_h) or
// from physical-grid models (vps, one per particle).
static int time_one(const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs, int Dmax,
                    const double *nodes_h, int ld_nodes, const std::vector<const float *> &vps, unsigned char *w,
                    const empso_tuning &tu, int warm, int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t st,
                    float *us_per_step) {
    if (!nodes_h && vps.size() != pp.size()) EMPSO_FAIL(EMPSO_EINVAL, "timing needs node values or models");
    forget_progress(w);
    Plan pl;
    pl.L = make_layout(pp, runs, Dmax, tu.bz, tu.tsteps);
    build_header(pl, w, pp, runs, vps, nodes_h, ld_nodes, Dmax, tu);
    const Layout &L = pl.L;
    EMPSO_HIP(hipMemcpyAsync(w, pl.host_hdr.data(), L.hdr_bytes, hipMemcpyHostToDevice, st));
    EMPSO_HIP(hipStreamSynchronize(st));
    const RunDesc *rd = reinterpret_cast<const RunDesc *>(w + L.runs_off);
    const int4 *td = reinterpret_cast<const int4 *>(w + L.tiles_off);
    k_zero<<<2048, 256, 0, st>>>(reinterpret_cast<float4 *>(w + L.state_off), (int64_t)(L.total - L.state_off) / 16);
    k_coef<<<dim3(512, (int)pp.size()), 256, 0, st>>>(reinterpret_cast<const CoefDesc *>(w + L.coef_off));
    for (int r = 0; r < warm; ++r)
        if (launch_tb(tu.tsteps, L.iso, rd, td, L.ntiles, 0, 0, st)) EMPSO_FAIL(EMPSO_ENOTSUP, "bad tuning");
    EMPSO_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r)
        if (launch_tb(tu.tsteps, L.iso, rd, td, L.ntiles, 0, 0, st)) EMPSO_FAIL(EMPSO_ENOTSUP, "bad tuning");
    EMPSO_HIP(hipEventRecord(e1, st));
    EMPSO_HIP(hipEventSynchronize(e1));
    EMPSO_HIP(hipGetLastError());
    float ms = 0.f;
    EMPSO_HIP(hipEventElapsedTime(&ms, e0, e1));
    *us_per_step = 1000.f * ms / (reps * tu.tsteps);
    return EMPSO_OK;
}

extern "C" int empso_time_tuning(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                                 const int32_t *pop, int32_t np, const double *nodes_h, int32_t ld_nodes, void *ws,
                                 size_t ws_bytes, const empso_tuning *tuning, int32_t reps, float *us_per_step,
                                 empso_stream stream) {
    clear_error();
    if (!tuning || !us_per_step) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (reps < 1) EMPSO_FAIL(EMPSO_EINVAL, "reps must be >= 1");
    empso_tuning tu = *tuning;
    tu.use_graph = 0;
    if (!valid_tuning(tu)) EMPSO_FAIL(EMPSO_ENOTSUP, "unsupported tuning");
    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    int Dmax;
    int rc = batch_prepare(probs, nprob, obs_d, pop, np, nodes_h, ld_nodes, ws, ws_bytes, pp, runs, &Dmax);
    if (rc) return rc;
    hipEvent_t e0, e1;
    EMPSO_HIP(hipEventCreate(&e0));
    EMPSO_HIP(hipEventCreate(&e1));
    std::lock_guard<std::mutex> lk(g_plan_mu);
    rc = time_one(pp, runs, Dmax, nodes_h, ld_nodes, std::vector<const float *>(), reinterpret_cast<unsigned char *>(ws),
                  tu, 1, reps, e0, e1,
                  (hipStream_t)stream, us_per_step);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Time every tile height of kTuneBz (the first of each distinct tiling)
// and depth T = 1 .. 4 on a batch (a few launches each) and keep the fastest.
// The caller holds g_plan_mu.
static int pick_tuning(const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs, int Dmax,
                       const double *nodes_h, int ld_nodes, const std::vector<const float *> &vps,
                       unsigned char *w, hipStream_t st, int warm, int reps, double final_ms, empso_tuning *best,
                       float *best_us) {
    hipEvent_t e0, e1;
    EMPSO_HIP(hipEventCreate(&e0));
    EMPSO_HIP(hipEventCreate(&e1));

    std::vector<std::pair<float, empso_tuning>> timed;
    int rc = EMPSO_OK;
    for (int T = 1; T <= kMaxT && rc == EMPSO_OK; ++T) {
        std::vector<std::vector<int>> seen;    // strip heights of the tilings timed at this depth
        for (int bi = 0; bi < kNumTuneBz && rc == EMPSO_OK; ++bi) {
            // tile heights that give every grid of the batch the same strips
            // launch the same tiles: time the first of them only
            std::vector<int> sig;
            for (const empso_problem *p : pp) sig.push_back(strip_height(p, kTuneBz[bi], T));
            if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
            seen.push_back(sig);
            empso_tuning tu;
            empso_default_tuning(&tu);
            tu.bz = kTuneBz[bi];
            tu.tsteps = T;
            tu.use_graph = 0;
            float us = 0.f;
            rc = time_one(pp, runs, Dmax, nodes_h, ld_nodes, vps, w, tu, warm, reps, e0, e1, st, &us);
            if (rc == EMPSO_OK) timed.emplace_back(us, tu);
        }
    }
    // Second round: a few launches can rank tilings that lie within a few
    // percent of each other differently from a sustained run (clocks and
    // caches settle over many launches); the three fastest are timed again
    // over about final_ms of launches each, after as many untimed ones.
    if (rc == EMPSO_OK && final_ms > 0 && timed.size() > 1) {
        std::stable_sort(timed.begin(), timed.end(),
                         [](const std::pair<float, empso_tuning> &x, const std::pair<float, empso_tuning> &y) {
                             return x.first < y.first;
                         });
        const size_t nfin = std::min<size_t>(3, timed.size());
        for (size_t i = 0; i < nfin && rc == EMPSO_OK; ++i) {
            const empso_tuning tu = timed[i].second;
            const double launch_ms = 1e-3 * timed[i].first * tu.tsteps;
            const int n = (int)std::min(200.0, std::max(4.0, final_ms / std::max(launch_ms, 1e-3)));
            float us = 0.f;
            rc = time_one(pp, runs, Dmax, nodes_h, ld_nodes, vps, w, tu, n, n, e0, e1, st, &us);
            if (rc == EMPSO_OK) timed[i].first = us;
        }
        std::stable_sort(timed.begin(), timed.begin() + nfin,
                         [](const std::pair<float, empso_tuning> &x, const std::pair<float, empso_tuning> &y) {
                             return x.first < y.first;
                         });
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (timed.empty()) EMPSO_FAIL(EMPSO_ENOTSUP, "no tuning could be timed");
    *best = timed.front().second;
    if (best_us) *best_us = timed.front().first;
    return EMPSO_OK;
}

extern "C" int empso_autotune_fitness(const empso_problem *const *probs, int32_t nprob, const float *const *obs_d,
                                      const int32_t *pop, int32_t np, const double *nodes_h, int32_t ld_nodes,
                                      void *ws, size_t ws_bytes, empso_tuning *best, float *best_us_per_step,
                                      empso_stream stream) {
    clear_error();
    if (!best) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    std::vector<const empso_problem *> pp;
    std::vector<RunSpec> runs;
    int Dmax;
    int rc = batch_prepare(probs, nprob, obs_d, pop, np, nodes_h, ld_nodes, ws, ws_bytes, pp, runs, &Dmax);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    empso_tuning bt;
    rc = pick_tuning(pp, runs, Dmax, nodes_h, ld_nodes, std::vector<const float *>(),
                     reinterpret_cast<unsigned char *>(ws), (hipStream_t)stream, 2, 4, 1000.0, &bt, best_us_per_step);
    if (rc) return rc;
    bt.use_graph = 1;
    *best = bt;
    return EMPSO_OK;
}

// Tuning of a forward modelling (record mode, models given on the grid).
static int forward_autotune(const std::vector<const empso_problem *> &pp, const std::vector<RunSpec> &runs,
                            const std::vector<const float *> &vps, unsigned char *w, hipStream_t st,
                            empso_tuning *best) {
    const int rc = pick_tuning(pp, runs, pp[0]->D, nullptr, 0, vps, w, st, 1, 2, 0.0, best, nullptr);
    best->use_graph = 0;
    return rc;
}

// ---------------------------------------------------------------------------
// Misfit gradient (the local FWI that follows the global search, Testing
// approach section), by the discrete adjoint of the scheme with checkpoints.
//
// Dividing the update by C = (v dt)^2 makes its operator symmetric, so the
// adjoint psi runs the same damped scheme backwards in time with the residual
// r^k = u^k - d^k injected at the receivers:
//   (1+a) psi^k = 2 psi^{k+1} - (1-a) psi^{k+2} + C (Lap_h psi^{k+1} + r^k),
// k = nt-1 .. 1, psi^{nt} = psi^{nt+1} = 0, and
//   dJ/dC = sum_n psi^{n+1} [(1+a) u^{n+1} - 2 u^n + (1-a) u^{n-1}] / C^2
// = sum_m u^m L^m / C after a summation by parts (u^0 = u^{-1} = 0 and
// psi^{nt} = psi^{nt+1} = 0 leave no boundary terms) and the adjoint
// recursion, with L^m = Lap_h psi^{m+1} + r^m the quantity each adjoint update
// multiplies by C,
//   dJ/dv = dJ/dC 2 v dt^2, folded from the padded grid onto the physical
// model (each padded point adds into the point it copies) and summed over
// shots. Both directions use the increment form of the fitness kernels. The
// forward pass keeps (u^{jK}, u^{jK-1}) every K steps; the backward pass
// restores each segment from its checkpoint, recomputes its K time levels and
// runs the adjoint through it, accumulating the gradient as it goes (and, if
// asked for, the illumination sum_n (u^n)^2 from the same recomputed levels).
// ---------------------------------------------------------------------------
namespace {

struct GradRun {
    float *fields;              // the run's fields, gfs floats apart
    const float *obs;           // [nt][nrec]
    double *acc;                // [nrec] sum of squared residuals over k >= 1 (l2)
    double *tsum;               // trace-normalised: [3][nrec] sums of d^2, d o, o^2, then the
                                // shot's floors wd, wo; else NULL
    float *ab;                  // trace-normalised: [3][nrec] adjoint-source factors a, b, 1/sd
    int srcS, srcC;             // stored row and column of the source
};

// Field slots of a run: nbuf buffers of K+2 segment levels each (with more
// than one segment, two buffers: the next segment is recomputed into one
// while the adjoint runs through the other), then the four contiguous fields
// that hold the forward state during the checkpointing pass and the adjoint's
// two pairs of levels afterwards, the gradient accumulator, the illumination
// accumulator, then two fields per checkpoint.
struct GradSlots {
    int K, ncheck, nbuf;
    int seg(int buf, int i) const { return buf * (K + 2) + i; }
    int adjp() const { return nbuf * (K + 2); }
    int gacc() const { return adjp() + 4; }
    int illum() const { return adjp() + 5; }
    int ck(int j, int which) const { return adjp() + 6 + 2 * j + which; }
    int total() const { return adjp() + 6 + 2 * ncheck; }
};

static int grad_interval(const empso_problem *p, int K) {
    if (K > 0) return K;
    return std::max(1, (int)std::ceil(std::sqrt(2.0 * std::max(1, p->g.nt - 1))));
}

static constexpr int kAdjT = 3;      // adjoint steps per launch of k_tba
static constexpr int kAdjBz = 40;    // its tile height (measured best with the overlapped recomputation)
// tile height and depth of the checkpointing pass (measured on 16 realistic
// shots: 0.489 s per gradient, against 0.526 s at the tiling the forward
// modelling's autotuner picks for the same shots, one step per launch)
static constexpr int kGradFwdBz = 20;
static constexpr int kGradFwdT = 2;
// tile height and depth of the segment recomputation, which shares the GPU
// with the adjoint (0: those of the checkpointing pass)
static constexpr int kGradRecBz = 40;
static constexpr int kGradRecT = 4;
// Adjoint of one run (shot) for the temporally blocked adjoint kernel.
struct AdjDesc {
    float *psi;                 // four contiguous fields; pair p holds (psi^{k+1}, psi^{k+2}) in fields p, 2 + p
    const float *C;             // coefficient field
    const float *seg;           // segment levels: u^m in field m - b + 1, gfs floats apart
    float *g;                   // imaging sum over m of u^m (Lap psi^{m+1} + r^m)
    const float *obs;           // [nt][nrec]
    double *acc;                // l2: [nrec] sums of squared residuals
    const float *ab;            // trace-normalised: [3][nrec] adjoint-source factors a, b, 1/sd; else NULL
    const float *ax, *az, *zoma, *zinv;
    const int *recmap;
    size_t gfs;
    int Nz, Nx, S, nrec, recS, zlo, zhi;
    unsigned fbytes;
    float cz1, cz2, cz3, cz4, cx1, cx2, cx3, cx4;
};

// T adjoint steps k, k-1, .., k-T+1 of every tile, all levels in registers:
// the same march as the fitness kernel k_tb with psi in the role of u, level
// l computing psi^{k-l} from psi^{k-l+1} and psi^{k-l+2}, and the adjoint
// source r^{k-l} (the residual at the receivers, or the trace-normalised
// misfit's derivative) added to the Laplacian on the receiver row in place of
// the Ricker source. The imaging sum takes u^{k-l} L at every point, with L =
// Lap psi^{k-l+1} + r^{k-l} the quantity the update multiplies by C: the
// adjoint recursion gives (1+a)(psi^m - psi^{m+1}) - (1-a)(psi^{m+1} - psi^{m+2})
// = C L exactly, so the sum is dJ/dC times C (dJ/dv = 2 sum / v). A row's T
// terms are added by the levels in time order (level 0 starts from the sum
// read from HBM); between levels the partial sums wait in an LDS ring of 10
// rows indexed by the step within the 10-step block, so every ring address is
// known at compile time (4 (T - 1) < 10). The residuals of the T levels at
// the receiver row are formed before the march and parked in LDS; the tile
// that owns the receiver row adds the squared l2 residuals to the misfit.
// u^{k-l} comes from the segment's stored levels. Stores, damping forms and
// the zero ring work as in k_tb.
template <int T, bool ISO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_tba(const AdjDesc *__restrict__ descs,
        const int4 *__restrict__ tiles, int ntiles, int k, int b, int par) {
    constexpr int NS = kQueue;
    constexpr int FILL = 8 * (T - 1);
    constexpr int TQ = T > 1 ? T - 1 : 1;
    static_assert(4 * (T - 1) < NS, "the imaging ring holds 10 rows");
    __shared__ float4 sres[4][T + 1][64];
    __shared__ float4 sg[4][NS][64];
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int wv = (int)(threadIdx.x >> 6);
    const int tix = __builtin_amdgcn_readfirstlane(lb * 4 + wv);
    if (tix >= ntiles) return;
    const int lane = threadIdx.x & 63;
    const int4 t = tiles[tix];
    const AdjDesc R = descs[t.x];
    const int S = R.S;
    const int bot = R.Nz + kRing;
    const rsrc_t F = make_rsrc(R.psi, 4u * R.fbytes);
    const int fb = (int)R.fbytes;
    const int uin = par ? fb : 0, vin = par ? 3 * fb : 2 * fb;
    const int uout = par ? 0 : fb, vout = par ? 2 * fb : 3 * fb;
    const rsrc_t Cf = make_rsrc(R.C, R.fbytes);
    const rsrc_t Gf = make_rsrc(R.g, R.fbytes);
    rsrc_t Uf[T];
#pragma unroll
    for (int l = 0; l < T; ++l) Uf[l] = make_rsrc(R.seg + (size_t)(k - l - b + 1) * R.gfs, R.fbytes);
    const int c = t.z + 4 * lane;
    const int cc = min(c, S - 4);
    const int J0 = c - kRing;
    const bool own = (lane >= T) && (lane < 64 - T);
    const int s0 = t.y;
    const int s1 = min(t.w, bot);
    const int lcol = 4 * cc;
    const int rowb = 4 * S;

    float axk[4], xoma[4], xinv[4];
    bool xdamp = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int J = J0 + q;
        axk[q] = (J >= 0 && J < R.Nx) ? gld(R.ax + J) : 0.0f;
        xoma[q] = 1.0f - axk[q];
        xinv[q] = __builtin_amdgcn_rcpf(1.0f + axk[q]);
        xdamp |= axk[q] != 0.0f;
    }
    const bool tile_xdamp = __any(xdamp);

    // adjoint sources of the T levels on the receiver row
    const bool rec_owner = own && R.recS >= s0 && R.recS < s1;
    sres[wv][T][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int l = 0; l < T; ++l) {
        const int m = k - l;
        const float4 u4 = bld4(Uf[l], R.recS * rowb + lcol);
        const float uu[4] = {u4.x, u4.y, u4.z, u4.w};
        float rr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int J = J0 + q;
            rr[q] = 0.0f;
            const int r = (J >= 0 && J < R.Nx) ? gld(R.recmap + J) : -1;
            if (r >= 0) {
                const float ob = gld(R.obs + (size_t)m * R.nrec + r);
                if (R.ab) {
                    rr[q] = fmaf(gld(R.ab + r), uu[q], -gld(R.ab + R.nrec + r) * ob) * gld(R.ab + 2 * R.nrec + r);
                } else {
                    rr[q] = uu[q] - ob;
                    if (rec_owner) gst(R.acc + r, gld(R.acc + r) + (double)rr[q] * (double)rr[q]);
                }
            }
        }
        sres[wv][l][lane] = make_float4(rr[0], rr[1], rr[2], rr[3]);
    }

    const int rs = s0 - 4 * (T - 1);
    float4 q0[NS], qu[TQ][NS], vq, cq[T], ukq[T], gq;
#pragma unroll
    for (int j = 0; j < 9; ++j) q0[j] = bld4(F, uin + (rs - 4 + j) * rowb + lcol);
    vq = bld4(F, vin + rs * rowb + lcol);
#pragma unroll
    for (int l = 0; l < T; ++l) {
        cq[l] = bld4(Cf, (rs - 4 * l) * rowb + lcol);
        ukq[l] = bld4(Uf[l], (rs - 4 * l) * rowb + lcol);
    }
    gq = bld4(Gf, rs * rowb + lcol);
#pragma unroll
    for (int l = 0; l < TQ; ++l) {
#pragma unroll
        for (int j = 0; j < NS; ++j) qu[l][j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    auto step = [&](const int kk, const int r1, auto mode_tag) __attribute__((always_inline)) {
        constexpr int mode = decltype(mode_tag)::value;
        q0[(kk + 9) % NS] = bld4(F, uin + (r1 + 5) * rowb + lcol);
        float4 un = make_float4(0.f, 0.f, 0.f, 0.f), ue = un, gout = un;
#pragma unroll
        for (int l = 0; l < T; ++l) {
            const float4 *src = (l == 0) ? q0 : qu[l > 0 ? l - 1 : 0];
            const float4 ce = src[(kk + 4) % NS];
            const float4 p1 = src[(kk + 3) % NS], m1 = src[(kk + 5) % NS];
            const float4 p2 = src[(kk + 2) % NS], m2 = src[(kk + 6) % NS];
            const float4 p3 = src[(kk + 1) % NS], m3 = src[(kk + 7) % NS];
            const float4 p4 = src[(kk + 0) % NS], m4 = src[(kk + 8) % NS];
            const float4 pv = (l == 0) ? vq : ((l == 1) ? q0 : qu[l > 1 ? l - 2 : 0])[kk % NS];
            const float4 C4 = cq[l];
            const float4 U4 = ukq[l];
            const int r = r1 - 4 * l;
            cq[l] = bld4(Cf, (r + 1) * rowb + lcol);
            ukq[l] = bld4(Uf[l], (r + 1) * rowb + lcol);
            if (l == 0) vq = bld4(F, vin + (r1 + 1) * rowb + lcol);
            const float v[12] = {from_lane_below(ce.x), from_lane_below(ce.y),
                                 from_lane_below(ce.z), from_lane_below(ce.w),
                                 ce.x, ce.y, ce.z, ce.w,
                                 from_lane_above(ce.x), from_lane_above(ce.y),
                                 from_lane_above(ce.z), from_lane_above(ce.w)};
            const float pz1[4] = {p1.x, p1.y, p1.z, p1.w}, mz1[4] = {m1.x, m1.y, m1.z, m1.w};
            const float pz2[4] = {p2.x, p2.y, p2.z, p2.w}, mz2[4] = {m2.x, m2.y, m2.z, m2.w};
            const float pz3[4] = {p3.x, p3.y, p3.z, p3.w}, mz3[4] = {m3.x, m3.y, m3.z, m3.w};
            const float pz4[4] = {p4.x, p4.y, p4.z, p4.w}, mz4[4] = {m4.x, m4.y, m4.z, m4.w};
            const float pvv[4] = {pv.x, pv.y, pv.z, pv.w};
            const float Cv[4] = {C4.x, C4.y, C4.z, C4.w};
            const float Uv[4] = {U4.x, U4.y, U4.z, U4.w};
            const int rz = min(max(r - kRing, 0), R.Nz - 1);
            const float azr = (mode == 3) ? sld(R.az + rz) : 0.0f;
            const float zo = (mode == 2) ? sld(R.zoma + rz) : 1.0f;
            const float zi = (mode == 2) ? sld(R.zinv + rz) : 1.0f;
            const float4 rs4 = sres[wv][(r == R.recS) ? l : T][lane];
            const float rsv[4] = {rs4.x, rs4.y, rs4.z, rs4.w};
            // imaging partial sum of this row: from HBM for the first level,
            // else from the ring slot the previous level left it in
            const float4 gp = (l == 0) ? gq : sg[wv][((kk - 4 * l) % NS + NS) % NS][lane];
            const float gpv[4] = {gp.x, gp.y, gp.z, gp.w};
            float uo[4], go[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float u = v[4 + q];
                float lap;
                if (ISO) {
                    lap = R.cz4 * ((pz4[q] + mz4[q]) + (v[0 + q] + v[8 + q]));
                    lap = fmaf(R.cz3, fmaf(-kFold3, u, (pz3[q] + mz3[q]) + (v[1 + q] + v[7 + q])), lap);
                    lap = fmaf(R.cz2, fmaf(-4.0f, u, (pz2[q] + mz2[q]) + (v[2 + q] + v[6 + q])), lap);
                    lap = fmaf(R.cz1, fmaf(-4.0f, u, (pz1[q] + mz1[q]) + (v[3 + q] + v[5 + q])), lap);
                } else {
                    lap = R.cz4 * (pz4[q] + mz4[q]);
                    lap = fmaf(R.cz3, fmaf(-kFold3Axis, u, pz3[q] + mz3[q]), lap);
                    lap = fmaf(R.cz2, fmaf(-2.0f, u, pz2[q] + mz2[q]), lap);
                    lap = fmaf(R.cz1, fmaf(-2.0f, u, pz1[q] + mz1[q]), lap);
                    lap = fmaf(R.cx4, v[0 + q] + v[8 + q], lap);
                    lap = fmaf(R.cx3, fmaf(-kFold3Axis, u, v[1 + q] + v[7 + q]), lap);
                    lap = fmaf(R.cx2, fmaf(-2.0f, u, v[2 + q] + v[6 + q]), lap);
                    lap = fmaf(R.cx1, fmaf(-2.0f, u, v[3 + q] + v[5 + q]), lap);
                }
                lap += rsv[q];
                const float dp = u - pvv[q];
                float d;
                if constexpr (mode == 0) {
                    d = fmaf(Cv[q], lap, dp);
                } else if constexpr (mode == 1) {
                    d = fmaf(Cv[q], lap, xoma[q] * dp) * xinv[q];
                } else if constexpr (mode == 2) {
                    d = fmaf(Cv[q], lap, zo * dp) * zi;
                } else {
                    const float a = azr + axk[q];
                    const float inv = __builtin_amdgcn_rcpf(1.0f + a);
                    d = fmaf(Cv[q], lap, (1.0f - a) * dp) * inv;
                }
                uo[q] = u + d;
                go[q] = fmaf(Uv[q], lap, gpv[q]);
            }
            const float4 g4 = make_float4(go[0], go[1], go[2], go[3]);
            if (l < T - 1)
                sg[wv][((kk - 4 * l) % NS + NS) % NS][lane] = g4;
            else
                gout = g4;
            if (l == 0) gq = bld4(Gf, (r1 + 1) * rowb + lcol);
            un = make_float4(uo[0], uo[1], uo[2], uo[3]);
            ue = ce;
            if (l < T - 1) qu[l][(kk + 8) % NS] = un;
        }
        const int rT = r1 - 4 * (T - 1);
        const bool ok = own && (rT >= s0) && (rT < s1);
        const int o = rT * rowb + lcol;
        bst4(F, ok ? uout + o : kDrop, un);
        bst4(F, ok ? vout + o : kDrop, ue);
        bst4(Gf, ok ? o : kDrop, gout);
    };
    auto step_any = [&](const int kk, const int r1) __attribute__((always_inline)) {
        const bool zrow = r1 - 4 * (T - 1) < R.zlo || r1 >= R.zhi;
        if (tile_xdamp) {
            if (zrow)
                step(kk, r1, std::integral_constant<int, 3>{});
            else
                step(kk, r1, std::integral_constant<int, 1>{});
        } else {
            if (zrow)
                step(kk, r1, std::integral_constant<int, 2>{});
            else
                step(kk, r1, std::integral_constant<int, 0>{});
        }
    };
    const int nit = FILL + (s1 - s0);
    for (int j = 0; j < nit; j += NS) {
#pragma unroll
        for (int kk = 0; kk < NS; ++kk) step_any(kk, rs + j + kk);
    }
}

__global__ void k_gcopy(const GradRun *__restrict__ runs, size_t gfs, int src, int dst) {
    const GradRun R = runs[blockIdx.y];
    const float4 *a = reinterpret_cast<const float4 *>(R.fields + (size_t)src * gfs);
    float4 *b = reinterpret_cast<float4 *>(R.fields + (size_t)dst * gfs);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < gfs / 4; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// Illumination of one segment: acc += (u^k)^2 at every stored point of every
// run for k = lo + n - 1 down to lo (the adjoint's order of time steps), u^k
// in field slot first + k - lo.
__global__ void k_gillum(const GradRun *__restrict__ runs, size_t gfs, int first, int n, int acc) {
    const GradRun R = runs[blockIdx.y];
    const size_t n4 = gfs / 4;
    const float4 *u = reinterpret_cast<const float4 *>(R.fields + (size_t)first * gfs);
    float4 *a = reinterpret_cast<float4 *>(R.fields + (size_t)acc * gfs);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        float4 sum = a[i];
        for (int m = n - 1; m >= 0; --m) {
            const float4 x = u[(size_t)m * n4 + i];
            sum.x = fmaf(x.x, x.x, sum.x);
            sum.y = fmaf(x.y, x.y, sum.y);
            sum.z = fmaf(x.z, x.z, sum.z);
            sum.w = fmaf(x.w, x.w, sum.w);
        }
        a[i] = sum;
    }
}

// Physical gradient: each physical point gathers the padded points that copy
// it (its own, plus the absorbing-layer strip or corner beyond an edge), over
// all runs in a fixed order, times 2 / v (the accumulator holds dJ/dC times C,
// and dJ/dv = dJ/dC 2 v dt^2 with C = (v dt)^2); the illumination accumulator
// (slot gacc + 1), if asked for, is gathered the same way.
__global__ void k_gfold(const GradRun *__restrict__ runs, int nruns, size_t gfs, int Nz, int Nx, int S, int gacc,
                        const float *vp, int nz, int nx, int nbl, float *grad, float *illum) {
    const int64_t n = (int64_t)nz * nx;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / nx), j = (int)(q - (int64_t)i * nx);
        const int I0 = i == 0 ? 0 : i + nbl, I1 = i == nz - 1 ? Nz - 1 : i + nbl;
        const int J0 = j == 0 ? 0 : j + nbl, J1 = j == nx - 1 ? Nx - 1 : j + nbl;
        double sum = 0.0, ill = 0.0;
        for (int r = 0; r < nruns; ++r) {
            const float *g = runs[r].fields + (size_t)gacc * gfs;
            const float *h = g + gfs;
            for (int I = I0; I <= I1; ++I)
                for (int J = J0; J <= J1; ++J) {
                    sum += (double)g[(size_t)(I + kRing) * S + J + kRing];
                    if (illum) ill += (double)h[(size_t)(I + kRing) * S + J + kRing];
                }
        }
        grad[q] = (float)(sum * 2.0 / (double)vp[q]);
        if (illum) illum[q] = (float)ill;
    }
}

// Adjoint source of the trace-normalised misfit, the sum over traces of
// m_r = 1/2 |d_r/sd_r - o_r/so_r|^2, sd_r = max(|d_r|, wd), so_r = max(|o_r|, wo),
// wd = EMPSO_TRACE_FLOOR |d_k| (k the largest modelled trace, lowest index
// on ties): dm/dd_r = (a_r d_r - b_r o_r) / sd_r with b_r = 1/so_r and
//   a_r = d_r.o_r / (|d_r|^2 so_r) above the floor (|d_r| > wd: d/|d| has the
//         Jacobian (I - e e^T)/|d|),
//   a_r = 1/wd at or below it (sd_r = wd),
// plus, for trace k, the dependence of wd on d_k: a_k += EMPSO_TRACE_FLOOR S
// with S = sum over the traces at or below the floor of
// dm_r/dwd = -(|d_r|^2/wd - d_r.o_r/so_r) / wd^2 (a fixed-order block sum).
// Zero when sd_r or so_r is zero. Kept as the three factors a, b, 1/sd, each
// of the size of 1/amplitude, so none overflows for data of any scale.
__global__ __launch_bounds__(256) void k_gab(const GradRun *__restrict__ runs, int nrec) {
    const GradRun R = runs[blockIdx.x];
    const double *dd = R.tsum, *dov = R.tsum + nrec, *oo = R.tsum + 2 * nrec;
    const double wd = trace_floor(dd, nrec), wo = trace_floor(oo, nrec);
    // largest modelled trace (lowest index on ties) and S
    __shared__ double rv[256], rs[256];
    __shared__ int ri[256];
    double bv = -1.0, sum = 0.0;
    int bi = nrec;
    for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
        if (dd[r] > bv) { bv = dd[r]; bi = r; }
        const double so = fmax(sqrt(oo[r]), wo);
        if (wd > 0.0 && sqrt(dd[r]) <= wd) sum -= (dd[r] / wd - (so > 0.0 ? dov[r] / so : 0.0)) / (wd * wd);
    }
    rv[threadIdx.x] = bv;
    ri[threadIdx.x] = bi;
    rs[threadIdx.x] = sum;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            const int o = threadIdx.x + k;
            if (rv[o] > rv[threadIdx.x] || (rv[o] == rv[threadIdx.x] && ri[o] < ri[threadIdx.x])) {
                rv[threadIdx.x] = rv[o];
                ri[threadIdx.x] = ri[o];
            }
            rs[threadIdx.x] += rs[o];
        }
        __syncthreads();
    }
    const int kmax = ri[0];
    const double S = rs[0];
    if (threadIdx.x == 0) {
        R.tsum[3 * nrec] = wd;
        R.tsum[3 * nrec + 1] = wo;
    }
    for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
        const double dn = sqrt(dd[r]), sd = fmax(dn, wd), so = fmax(sqrt(oo[r]), wo);
        float a = 0.0f, b = 0.0f, isd = 0.0f;
        if (sd > 0.0 && so > 0.0 && dd[r] < INFINITY) {
            double ad = dn > wd ? dov[r] / (dd[r] * so) : 1.0 / wd;
            if (r == kmax && wd > 0.0) ad += EMPSO_TRACE_FLOOR * S;
            a = (float)ad;
            b = (float)(1.0 / so);
            isd = (float)(1.0 / sd);
        }
        R.ab[r] = a;
        R.ab[nrec + r] = b;
        R.ab[2 * nrec + r] = isd;
    }
}

// J = sum over runs and receivers of the trace misfit: l2 1/2 (sum_{k>=1}
// r^k^2 + d^0^2) (u^0 = 0), or the trace-normalised misfit of the sums.
__global__ __launch_bounds__(256) void k_gmisfit(const GradRun *__restrict__ runs, int nruns, int nrec, int norm,
                                                 float *out) {
    double s = 0.0;
    for (int r = 0; r < nruns; ++r)
        for (int q = threadIdx.x; q < nrec; q += blockDim.x) {
            if (norm) {
                const double *t = runs[r].tsum;
                s += trace_normalised_misfit(t[q], t[nrec + q], t[2 * nrec + q], t[3 * nrec], t[3 * nrec + 1]);
            } else {
                const double d0 = runs[r].obs[q];
                s += 0.5 * (runs[r].acc[q] + d0 * d0);
            }
        }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)red[0];
}

struct GradLayout {
    GradSlots sl;
    size_t fb, runs_off, cd_off, adj_off, tiles_off, tiles1_off, fwd_runs_off, fwd_tiles_off, fwd_tiles1_off,
        rec_tiles_off, acc_off, tsum_off, ab_off, C_off, fields_off, total;
    int tile_cap;               // tile-table entries (all shots) for any tuning
};

static GradLayout grad_layout(const empso_problem *p, int K) {
    GradLayout L;
    L.sl.K = grad_interval(p, K);
    L.sl.ncheck = (std::max(1, p->g.nt - 1) - 1) / L.sl.K + 1;     // checkpoints at 0, K, .. <= nt - 2
    L.sl.nbuf = L.sl.ncheck > 1 ? 2 : 1;
    L.fb = field_bytes(p);
    size_t k = 0;
    auto take = [&](size_t b) { size_t r = k; k = align_up(k + b, 256); return r; };
    const int ns = p->g.nshots;
    L.runs_off = take(sizeof(GradRun) * ns);
    L.cd_off = take(sizeof(CoefDesc));
    L.adj_off = take(sizeof(AdjDesc) * ns * L.sl.nbuf);          // one table per segment buffer
    L.tile_cap = tile_capacity(p) * ns;
    L.tiles_off = take(sizeof(int4) * (size_t)L.tile_cap);
    L.tiles1_off = take(sizeof(int4) * (size_t)L.tile_cap);
    L.fwd_runs_off = take(sizeof(RunDesc) * ns * (1 + L.sl.nbuf));   // fitness-kernel passes: checkpointing,
                                                                     // then level keeping per segment buffer
    L.fwd_tiles_off = take(sizeof(int4) * (size_t)L.tile_cap);
    L.fwd_tiles1_off = take(sizeof(int4) * (size_t)L.tile_cap);
    L.rec_tiles_off = take(sizeof(int4) * (size_t)L.tile_cap);
    L.acc_off = take(sizeof(double) * (size_t)ns * p->g.nrec);
    const bool norm = p->g.misfit == EMPSO_MISFIT_TRACE_NORMALISED;
    L.tsum_off = take(norm ? sizeof(double) * (3 * (size_t)p->g.nrec + 2) * ns : 0);
    L.ab_off = take(norm ? sizeof(float) * 3 * (size_t)ns * p->g.nrec : 0);
    L.C_off = take(L.fb);
    L.fields_off = take(L.fb * (size_t)L.sl.total() * ns);
    L.total = k;
    return L;
}

}  // namespace

extern "C" size_t empso_gradient_workspace_bytes(const empso_problem *p, int32_t checkpoint_every) {
    if (!p || checkpoint_every < 0) return 0;
    return grad_layout(p, checkpoint_every).total;
}

extern "C" int empso_gradient(const empso_problem *p, const float *vp_d, const float *obs_d, float *grad_d,
                              float *misfit_d, float *illum_d, int32_t checkpoint_every, void *ws, size_t ws_bytes,
                              empso_stream stream) {
    clear_error();
    if (!p || !vp_d || !obs_d || !grad_d || !misfit_d || !ws) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (checkpoint_every < 0) EMPSO_FAIL(EMPSO_EINVAL, "checkpoint_every must be >= 0");
    if (p->g.nt < 2) EMPSO_FAIL(EMPSO_EINVAL, "the gradient needs nt >= 2");
    if (reinterpret_cast<uintptr_t>(ws) % 256) EMPSO_FAIL(EMPSO_EINVAL, "workspace must be 256-byte aligned");
    const GradLayout L = grad_layout(p, checkpoint_every);
    // level keeping addresses kMaxT + 2 consecutive fields through one buffer
    // resource with 32-bit byte offsets below 2^31 (kDrop must stay outside)
    if ((uint64_t)(kMaxT + 2) * L.fb >= ((uint64_t)1 << 31))
        EMPSO_FAIL(EMPSO_ENOTSUP, "grid too large for the gradient: a stored field takes %zu bytes (limit %llu)", L.fb,
                   (unsigned long long)(((uint64_t)1 << 31) / (kMaxT + 2)));
    if (ws_bytes < L.total) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> vh((size_t)p->g.nz * p->g.nx);
    EMPSO_HIP(hipMemcpyAsync(vh.data(), vp_d, vh.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    EMPSO_HIP(hipStreamSynchronize(st));
    for (size_t k = 0; k < vh.size(); ++k)
        if (!(vh[k] >= (float)p->g.vmin && vh[k] <= (float)p->g.vmax) || !std::isfinite(vh[k]))
            EMPSO_FAIL(EMPSO_ERANGE, "vp[%zu] = %g outside [%g, %g]", k, (double)vh[k], p->g.vmin, p->g.vmax);

    unsigned char *w = reinterpret_cast<unsigned char *>(ws);
    const int ns = p->g.nshots, nt = p->g.nt;
    const bool norm = p->g.misfit == EMPSO_MISFIT_TRACE_NORMALISED;
    const GradSlots &sl = L.sl;
    const size_t gfs = L.fb / sizeof(float);
    std::vector<GradRun> hr(ns);
    for (int s = 0; s < ns; ++s) {
        hr[s].fields = reinterpret_cast<float *>(w + L.fields_off + L.fb * (size_t)sl.total() * s);
        hr[s].obs = obs_d + (size_t)s * nt * p->g.nrec;
        hr[s].acc = reinterpret_cast<double *>(w + L.acc_off) + (size_t)s * p->g.nrec;
        hr[s].tsum = norm ? reinterpret_cast<double *>(w + L.tsum_off) + (3 * (size_t)p->g.nrec + 2) * s : nullptr;
        hr[s].ab = norm ? reinterpret_cast<float *>(w + L.ab_off) + (size_t)3 * s * p->g.nrec : nullptr;
        hr[s].srcS = p->srcI[s] + kRing;
        hr[s].srcC = p->srcJ[s] + kRing;
    }
    GradRun *runs = reinterpret_cast<GradRun *>(w + L.runs_off);
    // stream-ordered uploads (the caller's earlier work on st may still read
    // the workspace), waited for before the host copies go
    EMPSO_HIP(hipMemcpyAsync(runs, hr.data(), sizeof(GradRun) * ns, hipMemcpyHostToDevice, st));
    const float *Cf = reinterpret_cast<const float *>(w + L.C_off);
    const bool iso = p->g.dz == p->g.dx;

    // clear the fields and accumulators, then the coefficient field of vp
    const size_t zero_bytes = L.total - L.acc_off;
    k_zero<<<1024, 256, 0, st>>>(reinterpret_cast<float4 *>(w + L.acc_off), (int64_t)(zero_bytes / 16));
    CoefDesc cd = {};
    cd.C = reinterpret_cast<float *>(w + L.C_off);
    cd.vp = vp_d;
    cd.map = node_map(p);
    cd.nz = p->g.nz; cd.nx = p->g.nx; cd.nbl = p->g.nbl; cd.Nz = p->Nz; cd.Nx = p->Nx; cd.S = p->S;
    cd.dt = (float)p->g.dt;
    CoefDesc *cdd = reinterpret_cast<CoefDesc *>(w + L.cd_off);
    EMPSO_HIP(hipMemcpyAsync(cdd, &cd, sizeof(CoefDesc), hipMemcpyHostToDevice, st));
    EMPSO_HIP(hipStreamSynchronize(st));
    k_coef<<<dim3(1024, 1), 256, 0, st>>>(cdd);

    const int cblocks = (int)std::min<size_t>(4096, (gfs / 4 + 255) / 256);
    auto copy = [&](hipStream_t s, int src, int dst) {
        k_gcopy<<<dim3(cblocks, ns), 256, 0, s>>>(runs, gfs, src, dst);
    };

    // Tables of the checkpointing pass, which runs the fitness kernel on the
    // four state fields (no receivers with the l2 misfit; the trace sums of
    // the trace-normalised one), and of the blocked adjoint (k_tba, T adjoint
    // steps per launch; one descriptor table per segment buffer).
    const int Ta = kAdjT, bza = kAdjBz;
    std::vector<const empso_problem *> pp(1, p);
    std::vector<RunSpec> rsp;
    for (int s = 0; s < ns; ++s) rsp.push_back(RunSpec{p, 0, s, nullptr, nullptr});
    empso_tuning ftu;
    empso_default_tuning(&ftu);
    ftu.bz = kGradFwdBz;
    ftu.tsteps = kGradFwdT;
    const RunDesc *fruns = reinterpret_cast<const RunDesc *>(w + L.fwd_runs_off);
    const int4 *ftiles = reinterpret_cast<const int4 *>(w + L.fwd_tiles_off);
    const int4 *ftiles1 = reinterpret_cast<const int4 *>(w + L.fwd_tiles1_off);
    const int nft = tiles_of(p, ftu.bz, ftu.tsteps) * ns, nft1 = tiles_of(p, kTailBz, 1) * ns;
    const int rbz = kGradRecBz > 0 ? kGradRecBz : ftu.bz, rT = kGradRecT > 0 ? kGradRecT : ftu.tsteps;
    const int4 *rtiles = reinterpret_cast<const int4 *>(w + L.rec_tiles_off);
    const int nrt = tiles_of(p, rbz, rT) * ns;
    {
        // table 0: the checkpointing pass on the state fields; table 1 + buf:
        // level keeping on segment buffer buf
        std::vector<RunDesc> hf((size_t)ns * (1 + sl.nbuf));
        for (int q = 0; q <= sl.nbuf; ++q)
            for (int s = 0; s < ns; ++s) {
                RunDesc &d = hf[(size_t)q * ns + s];
                d = RunDesc{};
                float *f = hr[s].fields + (size_t)(q == 0 ? sl.adjp() : sl.seg(q - 1, 0)) * gfs;
                d.u[0] = f; d.u[1] = f + gfs; d.v[0] = f + 2 * gfs; d.v[1] = f + 3 * gfs;
                d.C = Cf;
                const bool sums = norm && q == 0;
                d.obs = sums ? hr[s].obs : nullptr;
                d.traces = nullptr;
                d.acc = sums ? hr[s].tsum : nullptr;    // [3][nrec] sums of d^2, d o, o^2
                d.wav = p->d_wav; d.az = p->d_az; d.ax = p->d_ax; d.recmap = p->d_recmap; d.reccol = p->d_reccol;
                d.zoma = p->d_zoma; d.zinv = p->d_zinv;
                d.Nz = p->Nz; d.Nx = p->Nx; d.S = p->S; d.nrec = p->g.nrec;
                d.recS = sums ? p->recI + kRing : -(1 << 30);   // otherwise no tile owns the receiver row
                d.zlo = p->zlo; d.zhi = p->zhi;
                d.norm = sums ? 1 : 0;
                d.srcS = hr[s].srcS; d.srcC = hr[s].srcC;
                d.nt = nt;
                d.fbytes = (unsigned)L.fb;
                d.c0 = p->c0;
                d.cz1 = p->cz[0]; d.cz2 = p->cz[1]; d.cz3 = p->cz[2]; d.cz4 = p->cz[3];
                d.cx1 = p->cx[0]; d.cx2 = p->cx[1]; d.cx3 = p->cx[2]; d.cx4 = p->cx[3];
                d.wscale = p->wscale;
            }
        std::vector<int4> ht(L.tile_cap), ht1(L.tile_cap);
        fill_tiles(ht.data(), pp, rsp, ftu.bz, ftu.tsteps);
        fill_tiles(ht1.data(), pp, rsp, kTailBz, 1);
        EMPSO_HIP(hipMemcpyAsync(w + L.fwd_runs_off, hf.data(), sizeof(RunDesc) * hf.size(), hipMemcpyHostToDevice,
                                 st));
        EMPSO_HIP(hipMemcpyAsync(w + L.fwd_tiles_off, ht.data(), sizeof(int4) * ht.size(), hipMemcpyHostToDevice, st));
        EMPSO_HIP(hipMemcpyAsync(w + L.fwd_tiles1_off, ht1.data(), sizeof(int4) * ht1.size(), hipMemcpyHostToDevice,
                                 st));
        std::vector<int4> htr(L.tile_cap);
        fill_tiles(htr.data(), pp, rsp, rbz, rT);
        EMPSO_HIP(hipMemcpyAsync(w + L.rec_tiles_off, htr.data(), sizeof(int4) * htr.size(), hipMemcpyHostToDevice,
                                 st));
        EMPSO_HIP(hipStreamSynchronize(st));        // the host tables may go once the copies are done
    }
    AdjDesc *adjd = reinterpret_cast<AdjDesc *>(w + L.adj_off);
    int4 *tdA = reinterpret_cast<int4 *>(w + L.tiles_off), *tdA1 = reinterpret_cast<int4 *>(w + L.tiles1_off);
    int ntA = 0, ntA1 = 0;
    {
        std::vector<AdjDesc> ha((size_t)ns * sl.nbuf);
        for (int buf = 0; buf < sl.nbuf; ++buf)
            for (int s = 0; s < ns; ++s) {
                AdjDesc &a = ha[(size_t)buf * ns + s];
                a.psi = hr[s].fields + (size_t)sl.adjp() * gfs;
                a.C = Cf;
                a.seg = hr[s].fields + (size_t)sl.seg(buf, 0) * gfs;
                a.g = hr[s].fields + (size_t)sl.gacc() * gfs;
                a.obs = hr[s].obs;
                a.acc = hr[s].acc;
                a.ab = hr[s].ab;
                a.ax = p->d_ax; a.az = p->d_az; a.zoma = p->d_zoma; a.zinv = p->d_zinv;
                a.recmap = p->d_recmap;
                a.gfs = gfs;
                a.Nz = p->Nz; a.Nx = p->Nx; a.S = p->S; a.nrec = p->g.nrec; a.recS = p->recI + kRing;
                a.zlo = p->zlo; a.zhi = p->zhi;
                a.fbytes = (unsigned)L.fb;
                a.cz1 = p->cz[0]; a.cz2 = p->cz[1]; a.cz3 = p->cz[2]; a.cz4 = p->cz[3];
                a.cx1 = p->cx[0]; a.cx2 = p->cx[1]; a.cx3 = p->cx[2]; a.cx4 = p->cx[3];
            }
        std::vector<int4> htA(L.tile_cap), htA1(L.tile_cap);
        fill_tiles(htA.data(), pp, rsp, bza, Ta);
        fill_tiles(htA1.data(), pp, rsp, kTailBz, 1);
        ntA = tiles_of(p, bza, Ta) * ns;
        ntA1 = tiles_of(p, kTailBz, 1) * ns;
        EMPSO_HIP(hipMemcpyAsync(adjd, ha.data(), sizeof(AdjDesc) * ha.size(), hipMemcpyHostToDevice, st));
        EMPSO_HIP(hipMemcpyAsync(tdA, htA.data(), sizeof(int4) * htA.size(), hipMemcpyHostToDevice, st));
        EMPSO_HIP(hipMemcpyAsync(tdA1, htA1.data(), sizeof(int4) * htA1.size(), hipMemcpyHostToDevice, st));
        EMPSO_HIP(hipStreamSynchronize(st));
    }
    auto launch_adj = [&](int T, int k, int b, int par, int buf) {
        const AdjDesc *ad = adjd + (size_t)buf * ns;
        const int4 *tt = T == 1 ? tdA1 : tdA;
        const int n_t = T == 1 ? ntA1 : ntA;
        int blocks = (n_t + 3) / 4;
        blocks = (blocks + 7) / 8 * 8;
#define EMPSO_TBA_CASE(TT)                                                                           \
        if (T == TT) {                                                                                \
            if (iso)                                                                                  \
                k_tba<TT, true><<<blocks, 256, 0, st>>>(ad, tt, n_t, k, b, par);                      \
            else                                                                                      \
                k_tba<TT, false><<<blocks, 256, 0, st>>>(ad, tt, n_t, k, b, par);                     \
        }
        EMPSO_TBA_CASE(1) EMPSO_TBA_CASE(2) EMPSO_TBA_CASE(3)
#undef EMPSO_TBA_CASE
    };

    // Checkpointing pass: the fitness kernel advances the state fields in
    // launches of T steps (single steps where a checkpoint is not a multiple
    // of T); after step jK the state pair holds (u^{jK}, u^{jK-1}), copied to
    // checkpoint j, for every jK <= nt - 2. The l2 misfit needs the pass up
    // to the last checkpoint only; the trace-normalised one needs whole
    // traces (their norms) before the adjoint starts, so it runs all steps
    // with the receivers sampled and then forms the adjoint-source weights.
    const int K = sl.K, last = sl.ncheck - 1;
    const int nfwd = norm ? nt - 1 : last * K;
    {
        int n = 0, par = 0;
        auto advance = [&](int n1) -> int {
            while (n < n1) {
                int rc;
                if (n + ftu.tsteps <= n1) {
                    rc = launch_tb(ftu.tsteps, iso, fruns, ftiles, nft, n, par, st);
                    n += ftu.tsteps;
                } else {
                    rc = launch_tb(1, iso, fruns, ftiles1, nft1, n, par, st);
                    n += 1;
                }
                if (rc) return rc;
                par ^= 1;
            }
            return EMPSO_OK;
        };
        for (int j = 1; j <= last; ++j) {
            const int rc = advance(j * K);
            if (rc) EMPSO_FAIL(rc, "launch failed");
            copy(st, sl.adjp() + par, sl.ck(j, 0));           // u^{jK} (field u of pair par)
            copy(st, sl.adjp() + 2 + par, sl.ck(j, 1));       // u^{jK-1} (field v of pair par)
        }
        const int rc = advance(nfwd);
        if (rc) EMPSO_FAIL(rc, "launch failed");
        if (norm) {
            k_sample<<<dim3(8, ns), 256, 0, st>>>(fruns, ns, nt - 1, par);     // the last sample
            k_gab<<<ns, 256, 0, st>>>(runs, p->g.nrec);
        }
        // the state fields become the adjoint's: psi^{nt} = psi^{nt+1} = 0
        for (int s = 0; s < ns; ++s)
            k_zero<<<256, 256, 0, st>>>(reinterpret_cast<float4 *>(hr[s].fields + (size_t)sl.adjp() * gfs),
                                        (int64_t)(4 * gfs / 4));
    }

    // Backward pass, segment by segment from the last: segment j covers
    // u^{jK-1} .. u^{e}, restored from checkpoint j (checkpoint 0 is the zero
    // initial state) and recomputed into slots 0 .. e - jK + 1 of buffer
    // j mod 2; the blocked adjoint carries its pair of psi levels across
    // segments. With two buffers, segment j - 1 is recomputed on a second
    // stream while the adjoint runs through segment j on the caller's stream:
    // each alone leaves most of the GPU idle with a few runs. Events order the
    // buffers' reuse: a recomputation waits for the adjoint that last read its
    // buffer, an adjoint for the recomputation of its segment.
    hipStream_t st2 = st;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // pass done, recomputed[2], adjoint done[2]
    struct EventGuard {
        hipEvent_t *e;
        ~EventGuard() {
            for (int k = 0; k < 5; ++k)
                if (e[k]) (void)hipEventDestroy(e[k]);
        }
    } guard{ev};
    if (sl.nbuf == 2) {
        const int rc = side_stream(&st2);
        if (rc) return rc;
        for (int k = 0; k < 5; ++k) EMPSO_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        EMPSO_HIP(hipEventRecord(ev[0], st));
        EMPSO_HIP(hipStreamWaitEvent(st2, ev[0], 0));
    }
    // a segment's levels by the fitness kernel keeping every level (launches of T
    // steps, single steps for the rest)
    auto recompute = [&](int j, int buf, hipStream_t s) -> int {
        const int b = j * K, e = std::min((j + 1) * K, nt - 1);
        copy(s, sl.ck(j, 1), sl.seg(buf, 0));
        copy(s, sl.ck(j, 0), sl.seg(buf, 1));
        const RunDesc *rr = fruns + (size_t)(1 + buf) * ns;
        for (int n = b; n < e;) {
            const int T = n + rT <= e ? rT : 1;
            const int rc = launch_tb_keep(T, iso, rr, T == 1 ? ftiles1 : rtiles, T == 1 ? nft1 : nrt, n, b, s);
            if (rc) return rc;
            n += T;
        }
        return EMPSO_OK;
    };
    int apar = 0;
    if (recompute(last, last % sl.nbuf, st)) EMPSO_FAIL(EMPSO_ENOTSUP, "launch failed");
    for (int j = last; j >= 0; --j) {
        const int b = j * K, e = std::min((j + 1) * K, nt - 1), buf = j % sl.nbuf;
        if (j > 0) {                                         // then nbuf == 2
            const int nb = (j - 1) % 2;
            if (j + 1 <= last) EMPSO_HIP(hipStreamWaitEvent(st2, ev[3 + nb], 0));
            if (recompute(j - 1, nb, st2)) EMPSO_FAIL(EMPSO_ENOTSUP, "launch failed");
            EMPSO_HIP(hipEventRecord(ev[1 + nb], st2));
        }
        if (j < last) EMPSO_HIP(hipStreamWaitEvent(st, ev[1 + buf], 0));
        for (int k = e; k >= b + 1; apar ^= 1) {
            const int T = (k - Ta + 1 >= b + 1) ? Ta : 1;
            launch_adj(T, k, b, apar, buf);
            k -= T;
        }
        // the illumination of u^{b+1} .. u^e (slots 2 .. e - b + 1), before the
        // buffer is released to the next recomputation
        if (illum_d) k_gillum<<<dim3(cblocks, ns), 256, 0, st>>>(runs, gfs, sl.seg(buf, 2), e - b, sl.illum());
        if (sl.nbuf == 2) EMPSO_HIP(hipEventRecord(ev[3 + buf], st));
    }
    const int64_t npts = (int64_t)p->g.nz * p->g.nx;
    k_gfold<<<(int)std::min<int64_t>(2048, (npts + 255) / 256), 256, 0, st>>>(
        runs, ns, gfs, p->Nz, p->Nx, p->S, sl.gacc(), vp_d, p->g.nz, p->g.nx, p->g.nbl, grad_d, illum_d);
    k_gmisfit<<<1, 256, 0, st>>>(runs, ns, p->g.nrec, norm ? 1 : 0, misfit_d);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}
