"""FP64 reference of the per-particle fitness evaluation (test infrastructure only).

The paper's fitness evaluation (Testing approach section; Results section) is:
control-node velocities are bilinearly interpolated onto the finite-difference
grid (the two-grid strategy), every shot is modelled with a finite-difference
scheme of second order in time and eighth order in space with a damping
absorbing layer of nbpml points and a Ricker source, the wavefield is sampled
at one receiver per surface grid column, and the modelled traces are scored
with the l2 norm against the observed traces, summed over shots.

Conventions the paper leaves open, and the reading taken here:
  * point (i, j) is at z = i*dz, x = j*dx; z points down; origin top-left.
    The padded grid adds nbl points on every side; beyond it u = 0.
  * the absorbing layer is the quadratic damping profile of Collino and
    Tsogka (2001): d(l) = d0 (l/nbl)^2 with d0 = 3 vmax ln(1/R) / (2 nbl h),
    l the depth into the layer in points; the x and z profiles add.
  * the source term enters the step n -> n+1 as wavelet[n]/(dz dx) at the
    source point; traces sample u^n for n = 0..nt-1; u^0 = u^{-1} = 0.
  * Ricker wavelet with peak frequency f0 and delay t0 = 1/f0.
  * misfit = 1/2 sum of squared residuals (the paper's l2 norm, squared and
    halved; the search only compares misfits, so any increasing transform
    leaves it unchanged). Optional variant (geometry key "misfit" =
    "trace_normalised"): every trace, one receiver of one shot over time, of
    the modelled and of the observed data is divided by its own l2 norm, or
    by a floor of 1e-4 times the largest trace norm of the same shot and side
    (modelled or observed) where that is larger (a zero trace stays zero),
    before that misfit. The paper states the plain l2 norm; the
    normalisation is the usual remedy for a source whose amplitude the
    modelling does not know, and the floor keeps traces with no arrival from
    being raised to full weight.
  * control nodes form a regular ncz x ncx grid whose corners are the corners
    of the physical grid; the padded layer copies the nearest physical value.
  * the paper's irregular node grid (Testing approach section: nodes built
    from a 1-D prior by resolution criteria it does not state, a water layer
    fixed by the prior) is read as a layered grid: depth levels, each with its
    own node x positions; linear along each level in x, then linear in z
    between the two levels around a point, constant beyond the first and last
    node of a level and above / below the first / last level; the top
    water_rows physical rows hold the water velocity.
"""
import ctypes
import math
import os
from concurrent.futures import ThreadPoolExecutor
from fractions import Fraction

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_forward_run.restype = ctypes.c_int
        lib.oracle_forward_run.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
            ctypes.c_double, ctypes.c_int, P(ctypes.c_double),
            ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double),
            ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double),
            P(ctypes.c_int), P(ctypes.c_double),
            P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double)]
        lib.oracle_gradient_run.restype = ctypes.c_int
        lib.oracle_gradient_run.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
            ctypes.c_double, ctypes.c_int, P(ctypes.c_double),
            ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double),
            ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double),
            P(ctypes.c_int), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double)]
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Stencil weights and stability
# ---------------------------------------------------------------------------

def fd_weights(M=4):
    """Exact central weights c_0..c_M of the second derivative, order 2M.

    Eighth order in space (Testing approach section; JSON key space_order = 8)
    means M = 4. For u''(0) h^2 ~ c_0 u(0) + sum_k c_k (u(kh) + u(-kh)), the
    Taylor expansion is matched through order 2M when
        c_0 + 2 sum_k c_k = 0,   2 sum_k c_k k^(2j) = (2j)! delta_{j,1}, j = 1..M.
    Solved in exact rationals (Gauss-Jordan on Fractions).
    Pinned by: the moment conditions themselves, exactness on polynomials,
    the published Fornberg (1988) table (tests/golden) and the symbol at pi.
    """
    n = M + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for j in range(n):
        A[j][0] = Fraction(1) if j == 0 else Fraction(0)
        for k in range(1, M + 1):
            A[j][k] = Fraction(2 * k ** (2 * j))
        b[j] = Fraction(math.factorial(2 * j)) if j == 1 else Fraction(0)
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        p = A[col][col]
        A[col] = [v / p for v in A[col]]
        b[col] = b[col] / p
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [vr - f * vc for vr, vc in zip(A[r], A[col])]
                b[r] = b[r] - f * b[col]
    return b


def symbol(weights, theta):
    """Fourier symbol s(theta) = c_0 + 2 sum_k c_k cos(k theta) of the 1-D stencil."""
    w = [float(c) for c in weights]
    theta = np.asarray(theta, dtype=np.float64)
    s = np.full_like(theta, w[0])
    for k in range(1, len(w)):
        s = s + 2.0 * w[k] * np.cos(k * theta)
    return s


def stable_dt(vmax, dz, dx, weights=None):
    """Largest stable leapfrog time step for the 2-D stencil at velocity vmax.

    Von Neumann analysis of u^{n+1} - 2u^n + u^{n-1} = (v dt)^2 Lap_h u^n gives
    stability iff (v dt)^2 S (1/dz^2 + 1/dx^2) <= 4, S = max_theta |s(theta)|.
    S is found by brute force on a dense grid of theta that contains pi.
    Pinned by: the closed form S = 2048/315 and a growth/boundedness run of
    the time loop just below and just above the limit.
    """
    if weights is None:
        weights = fd_weights(4)
    theta = np.linspace(0.0, np.pi, 200001)
    S = float(np.max(np.abs(symbol(weights, theta))))
    return 2.0 / (vmax * math.sqrt(S * (1.0 / dz ** 2 + 1.0 / dx ** 2)))


def n_steps(tmax, dt):
    """Number of samples nt = floor(tmax/dt) + 1 (t = 0 included)."""
    return int(math.floor(tmax / dt + 1e-9)) + 1


# ---------------------------------------------------------------------------
# Source, damping, model
# ---------------------------------------------------------------------------

def ricker(f0, dt, nt, t0=None):
    """Ricker wavelet w(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0.

    Paper: Ricker source (Testing approach section; JSON key f0). t0 = 1/f0.
    Pinned by: peak 1 at t0, zeros at t0 +- 1/(pi f0 sqrt 2), zero integral.
    """
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (np.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def damping_profile(nz, nx, nbl, dz, dx, vmax, R=1e-3):
    """Damping coefficient d(I, J) on the padded grid [nz+2nbl][nx+2nbl] (1/s).

    Paper: absorbing layer of nbpml points (JSON key nbpml); profile not given.
    Reading: quadratic profile d0 (l/nbl)^2, d0 = 3 vmax ln(1/R)/(2 nbl h),
    l = depth into the layer in points, z and x parts added.
    Pinned as a physical absorber (tests/test_oracle_absorber.py): on a 1 km
    grid with a 40-point layer the records differ from those of a grid too
    large for echoes by under 3 % (1.9 %), the difference grows as the layer
    thins, and wrong profiles (x damping only, a peak ten times too weak or too
    strong) exceed that.
    """
    Nz, Nx = nz + 2 * nbl, nx + 2 * nbl
    out = np.zeros((Nz, Nx), dtype=np.float64)
    if nbl == 0:
        return out
    d0z = 3.0 * vmax * math.log(1.0 / R) / (2.0 * nbl * dz)
    d0x = 3.0 * vmax * math.log(1.0 / R) / (2.0 * nbl * dx)
    I = np.arange(Nz)
    J = np.arange(Nx)
    lz = np.maximum(0, np.maximum(nbl - I, I - (Nz - 1 - nbl)))
    lx = np.maximum(0, np.maximum(nbl - J, J - (Nx - 1 - nbl)))
    dzp = d0z * (lz / nbl) ** 2
    dxp = d0x * (lx / nbl) ** 2
    out[:, :] = dzp[:, None] + dxp[None, :]
    return out


def vp_from_nodes(nodes, ncz, ncx, nz, nx):
    """Bilinear two-grid interpolation of control-node velocities onto the FD grid.

    Paper: the coarse-grid nodes are bilinearly interpolated to the FD grid
    (Testing approach section, two-grid strategy). Reading for a regular node
    grid: node (a, b) sits at grid coordinates (a (nz-1)/(ncz-1), b (nx-1)/(ncx-1));
    nodes are stored row-major [a][b]; the last cell is closed.
    Pinned by: exact reproduction of bilinear functions, node values at node
    sites, and the convex-combination bound.
    """
    g = np.asarray(nodes, dtype=np.float64).reshape(ncz, ncx)
    si = np.arange(nz, dtype=np.float64) * (ncz - 1) / (nz - 1)
    sj = np.arange(nx, dtype=np.float64) * (ncx - 1) / (nx - 1)
    a = np.minimum(np.floor(si).astype(np.int64), ncz - 2)
    b = np.minimum(np.floor(sj).astype(np.int64), ncx - 2)
    t = (si - a)[:, None]
    u = (sj - b)[None, :]
    A, B = a[:, None], b[None, :]
    return ((1 - t) * (1 - u) * g[A, B] + (1 - t) * u * g[A, B + 1]
            + t * (1 - u) * g[A + 1, B] + t * u * g[A + 1, B + 1])


def vp_from_levels(nodes, node_z, level_nodes, node_x, nz, nx, dz, dx, water_rows=0, v_water=1500.0):
    """Two-grid interpolation from a layered node grid (the reading of the
    paper's irregular grid stated in the module header).

    node_z[L] level depths (m, increasing); level a holds level_nodes[a] nodes
    at x positions node_x (m, increasing within a level, levels concatenated,
    the same order as `nodes`). Point (i, j) at z = i dz, x = j dx:
      v_a(x) = linear interpolation of level a's nodes at x (held constant
               beyond its first and last node),
      v(z, x) = (1 - t) v_a(x) + t v_{a+1}(x) for z_a <= z <= z_{a+1},
               t = (z - z_a)/(z_{a+1} - z_a); v_0 above the first level and
               v_{L-1} below the last one;
    rows i < water_rows hold v_water. Plain loops over grid points.
    Pinned by: bilinear functions sampled on a rectilinear layout are
    reproduced exactly, node values at node sites, linear interpolation along
    a level row and across levels at a column (np.interp), the water rows and
    the convex-combination bound.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    node_z = np.asarray(node_z, dtype=np.float64)
    node_x = np.asarray(node_x, dtype=np.float64)
    L = len(node_z)
    starts = np.concatenate([[0], np.cumsum(level_nodes)]).astype(np.int64)
    if nodes.size != starts[-1] or node_x.size != starts[-1]:
        raise ValueError("nodes and node_x must hold sum(level_nodes) values")

    def along(a, x):
        xs = node_x[starts[a]:starts[a + 1]]
        vs = nodes[starts[a]:starts[a + 1]]
        if x <= xs[0]:
            return vs[0]
        if x >= xs[-1]:
            return vs[-1]
        b = 0
        while xs[b + 1] < x:
            b += 1
        u = (x - xs[b]) / (xs[b + 1] - xs[b])
        return (1.0 - u) * vs[b] + u * vs[b + 1]

    out = np.empty((nz, nx), dtype=np.float64)
    for i in range(nz):
        z = i * dz
        if i < water_rows:
            out[i, :] = v_water
            continue
        if z <= node_z[0]:
            a, t = 0, 0.0
        elif z >= node_z[-1]:
            a, t = L - 2, 1.0
        else:
            a = 0
            while node_z[a + 1] < z:
                a += 1
            t = (z - node_z[a]) / (node_z[a + 1] - node_z[a])
        for j in range(nx):
            x = j * dx
            out[i, j] = (1.0 - t) * along(a, x) + t * along(a + 1, x)
    return out


def pad_edge(vp, nbl):
    """Extend a physical-grid field into the absorbing layer by nearest-value copy."""
    return np.pad(np.asarray(vp, dtype=np.float64), nbl, mode="edge")


def point_weights(pos, dz, dx, nz, nx, nbl):
    """Bilinear weights of a (z, x) position on the padded grid: [(I, J, w), ...].

    On-grid positions give a single point of weight 1. Injection uses the same
    weights as sampling (injection is the transpose of sampling).
    """
    zi = pos[0] / dz
    xj = pos[1] / dx
    if abs(zi - round(zi)) < 1e-9:
        zi = float(round(zi))
    if abs(xj - round(xj)) < 1e-9:
        xj = float(round(xj))
    if not (0.0 <= zi <= nz - 1 and 0.0 <= xj <= nx - 1):
        raise ValueError("position outside the physical grid: %r" % (pos,))
    i0 = min(int(math.floor(zi)), nz - 1)
    j0 = min(int(math.floor(xj)), nx - 1)
    ti, tj = zi - i0, xj - j0
    pts = []
    for di, wi in ((0, 1.0 - ti), (1, ti)):
        for dj, wj in ((0, 1.0 - tj), (1, tj)):
            w = wi * wj
            if w != 0.0:
                pts.append((i0 + di + nbl, j0 + dj + nbl, w))
    return pts


# ---------------------------------------------------------------------------
# Forward modelling
# ---------------------------------------------------------------------------

def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def forward_run(vel_pad, damp, dz, dx, dt, nt, wavelet, src_pts, rec_pts, nrec,
                weights=None, u0=None, um1=None, want_final=False):
    """One forward run on a padded grid (see oracle_fd.c for the scheme).

    src_pts: [(I, J, w)]; rec_pts: [(I, J, w, r)] with r the receiver index.
    Returns traces[nt][nrec] (and u^{nt-1} when want_final).
    """
    lib = _load()
    if weights is None:
        weights = fd_weights(4)
    w5 = np.array([float(c) for c in weights], dtype=np.float64)
    vel = np.ascontiguousarray(vel_pad, dtype=np.float64)
    dmp = np.ascontiguousarray(damp, dtype=np.float64)
    Nz, Nx = vel.shape
    wav = None if wavelet is None else np.ascontiguousarray(wavelet, dtype=np.float64)
    sI = np.array([p[0] for p in src_pts], dtype=np.int32)
    sJ = np.array([p[1] for p in src_pts], dtype=np.int32)
    sw = np.array([p[2] for p in src_pts], dtype=np.float64)
    rI = np.array([p[0] for p in rec_pts], dtype=np.int32)
    rJ = np.array([p[1] for p in rec_pts], dtype=np.int32)
    rw = np.array([p[2] for p in rec_pts], dtype=np.float64)
    rid = np.array([p[3] for p in rec_pts], dtype=np.int32)
    traces = np.zeros((nt, max(nrec, 1)), dtype=np.float64)
    fin = np.zeros((Nz, Nx), dtype=np.float64) if want_final else None
    a0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    a1 = None if um1 is None else np.ascontiguousarray(um1, dtype=np.float64)
    nullD = ctypes.POINTER(ctypes.c_double)()
    rc = lib.oracle_forward_run(
        Nz, Nx, float(dz), float(dx), _dptr(w5), _dptr(vel), _dptr(dmp), float(dt), int(nt),
        nullD if wav is None else _dptr(wav),
        len(sI), _iptr(sI), _iptr(sJ), _dptr(sw),
        int(nrec), len(rI), _iptr(rI), _iptr(rJ), _dptr(rw), _iptr(rid),
        _dptr(traces), nullD if a0 is None else _dptr(a0), nullD if a1 is None else _dptr(a1),
        nullD if fin is None else _dptr(fin))
    if rc != 0:
        raise MemoryError("oracle_forward_run failed")
    traces = traces[:, :nrec]
    return (traces, fin) if want_final else traces


class Problem:
    """Geometry of one modelling problem (see workloads.configs for the keys).

    dt and nt are explicit: the caller chooses them (normally dt_frac times
    stable_dt(vmax) and n_steps(tmax, dt)).
    """

    def __init__(self, geom, dt=None, nt=None):
        self.g = geom
        self.nz, self.nx = int(geom["nz"]), int(geom["nx"])
        self.dz, self.dx = float(geom["dz"]), float(geom["dx"])
        self.nbl = int(geom["nbl"])
        self.vmax = float(geom["vmax"])
        if dt is None:
            dt = geom["dt_frac"] * stable_dt(self.vmax, self.dz, self.dx)
        if nt is None:
            nt = n_steps(geom["tmax"], dt)
        self.dt, self.nt = float(dt), int(nt)
        self.f0 = float(geom["f0"])
        self.src = [tuple(p) for p in geom["src"]]
        self.rec = [tuple(p) for p in geom["rec"]]
        self.ncz, self.ncx = int(geom.get("ncz", 0)), int(geom.get("ncx", 0))
        self.levels = None
        if geom.get("node_z") is not None:
            self.levels = (np.asarray(geom["node_z"], dtype=np.float64),
                           [int(n) for n in geom["level_nodes"]],
                           np.asarray(geom["node_x"], dtype=np.float64))
        self.misfit = geom.get("misfit", "l2")
        if self.misfit not in ("l2", "trace_normalised"):
            raise ValueError("misfit must be 'l2' or 'trace_normalised'")
        self.water_rows = int(geom.get("water_rows", 0))
        self.v_water = float(geom.get("v_water", 1500.0))
        self.R = float(geom.get("damp_R", 1e-3))
        self.damp = damping_profile(self.nz, self.nx, self.nbl, self.dz, self.dx, self.vmax, self.R)
        self.wavelet = ricker(self.f0, self.dt, self.nt)
        self.rec_pts = []
        for r, pos in enumerate(self.rec):
            for (I, J, w) in point_weights(pos, self.dz, self.dx, self.nz, self.nx, self.nbl):
                self.rec_pts.append((I, J, w, r))

    @property
    def nshots(self):
        return len(self.src)

    @property
    def D(self):
        return int(sum(self.levels[1])) if self.levels else self.ncz * self.ncx

    def model(self, nodes):
        """Physical-grid model of one particle (regular or layered node grid)."""
        if self.levels:
            z, n, x = self.levels
            return vp_from_levels(nodes, z, n, x, self.nz, self.nx, self.dz, self.dx,
                                  self.water_rows, self.v_water)
        vp = vp_from_nodes(nodes, self.ncz, self.ncx, self.nz, self.nx)
        if self.water_rows:
            vp[:self.water_rows, :] = self.v_water
        return vp

    @property
    def nrec(self):
        return len(self.rec)

    def run(self, vel_pad, shot):
        spts = point_weights(self.src[shot], self.dz, self.dx, self.nz, self.nx, self.nbl)
        return forward_run(vel_pad, self.damp, self.dz, self.dx, self.dt, self.nt,
                           self.wavelet, spts, self.rec_pts, self.nrec)


def gradient_run(prob, vel_pad, shot, d_obs_shot):
    """Misfit of one shot and its gradient with respect to the padded-grid
    velocity (discrete adjoint, oracle_fd.c). Returns (J, grad[Nz][Nx])."""
    lib = _load()
    w5 = np.array([float(c) for c in fd_weights(4)], dtype=np.float64)
    vel = np.ascontiguousarray(vel_pad, dtype=np.float64)
    dmp = np.ascontiguousarray(prob.damp, dtype=np.float64)
    Nz, Nx = vel.shape
    spts = point_weights(prob.src[shot], prob.dz, prob.dx, prob.nz, prob.nx, prob.nbl)
    sI = np.array([p[0] for p in spts], dtype=np.int32)
    sJ = np.array([p[1] for p in spts], dtype=np.int32)
    sw = np.array([p[2] for p in spts], dtype=np.float64)
    rp = prob.rec_pts
    rI = np.array([p[0] for p in rp], dtype=np.int32)
    rJ = np.array([p[1] for p in rp], dtype=np.int32)
    rw = np.array([p[2] for p in rp], dtype=np.float64)
    rid = np.array([p[3] for p in rp], dtype=np.int32)
    dob = np.ascontiguousarray(d_obs_shot, dtype=np.float64)
    wav = np.ascontiguousarray(prob.wavelet, dtype=np.float64)
    grad = np.zeros((Nz, Nx), dtype=np.float64)
    J = ctypes.c_double()
    rc = lib.oracle_gradient_run(Nz, Nx, float(prob.dz), float(prob.dx), _dptr(w5), _dptr(vel), _dptr(dmp),
                                 float(prob.dt), int(prob.nt), _dptr(wav), len(sI), _iptr(sI), _iptr(sJ),
                                 _dptr(sw), int(prob.nrec), len(rI), _iptr(rI), _iptr(rJ), _dptr(rw),
                                 _iptr(rid), _dptr(dob), _dptr(grad), ctypes.byref(J))
    if rc != 0:
        raise MemoryError("oracle_gradient_run failed")
    return J.value, grad


def unpad_adjoint(g_pad, nbl):
    """Transpose of pad_edge: every padded point adds into the physical point
    it copies."""
    g = np.array(g_pad, dtype=np.float64)
    if nbl == 0:
        return g
    g[nbl, :] += g[:nbl, :].sum(axis=0)
    g[-nbl - 1, :] += g[-nbl:, :].sum(axis=0)
    g = g[nbl:-nbl, :]
    g[:, nbl] += g[:, :nbl].sum(axis=1)
    g[:, -nbl - 1] += g[:, -nbl:].sum(axis=1)
    return g[:, nbl:-nbl]


def normalised_adjoint_data(d, o):
    """Data o' of one shot ([nt][nrec]) for which the l2 residual d - o' is
    the derivative of the trace-normalised misfit, the sum over traces of
    m_r = 1/2 |d_r/s_r - o_hat_r|^2 (s_r = max(|d_r|, w), w the modelled
    floor, o_hat the normalised observed traces), with respect to the
    modelled traces d:
      * above the floor (|d_r| > w) d_r/|d_r| has the Jacobian
        (I - e e^T)/|d_r|, e = d_r/|d_r|: dm_r/dd_r = (I - e e^T)(e - o_hat_r)/|d_r|;
      * at or below it s_r = w: dm_r/dd_r = (d_r/w - o_hat_r)/w, and m_r also
        depends on w = TRACE_FLOOR |d_k| (k the largest modelled trace) with
        dm_r/dw = -d_r . (d_r/w - o_hat_r) / w^2, which adds
        TRACE_FLOOR (sum of those) d_k/|d_k| to the derivative for trace k.
    o' = d - dm/dd."""
    d = np.asarray(d, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    w = trace_floor(d)
    oh = normalise_traces(o, trace_floor(o))
    norms = np.sqrt(np.sum(d * d, axis=0))
    g = np.zeros_like(d)
    dm_dw = 0.0
    for r in range(d.shape[1]):
        x, y, n = d[:, r], oh[:, r], float(norms[r])
        if n > w:
            e = x / n
            g[:, r] = ((e - y) - e * np.dot(e, e - y)) / n
        elif w > 0:
            g[:, r] = (x / w - y) / w
            dm_dw -= np.dot(x, x / w - y) / w ** 2
    if w > 0:
        k = int(np.argmax(norms))
        g[:, k] += TRACE_FLOOR * dm_dw * d[:, k] / norms[k]
    return d - g


def gradient(prob, vp, d_obs, shots=None, threads=None):
    """Misfit summed over shots and its gradient with respect to the physical
    model vp[nz][nx] (Testing approach section: the local FWI that follows
    the global search needs the gradient of the same misfit). The exact
    gradient of the discrete misfit: pinned against central finite
    differences of forward_shots / misfit. For the trace-normalised misfit
    the adjoint is driven by the misfit's derivative with respect to the
    modelled traces, which needs the whole traces first (a forward pass)."""
    shots = list(range(prob.nshots)) if shots is None else list(shots)
    vel = pad_edge(vp, prob.nbl)
    norm = prob.misfit == "trace_normalised"

    def one(s):
        if not norm:
            return gradient_run(prob, vel, s, d_obs[s])
        tr = prob.run(vel, s)
        _, g = gradient_run(prob, vel, s, normalised_adjoint_data(tr, d_obs[s]))
        return misfit_normalised(tr, d_obs[s]), g

    with ThreadPoolExecutor(_workers(threads)) as ex:
        out = list(ex.map(one, shots))
    J = float(sum(o[0] for o in out))
    g_pad = np.sum([o[1] for o in out], axis=0)
    return J, unpad_adjoint(g_pad, prob.nbl)


def _workers(threads):
    return threads or min(16, os.cpu_count() or 1)


def forward_shots(prob, vp, shots=None, threads=None):
    """Traces [nshots][nt][nrec] (float64) of a physical-grid model vp[nz][nx]."""
    shots = list(range(prob.nshots)) if shots is None else list(shots)
    vel = pad_edge(vp, prob.nbl)
    with ThreadPoolExecutor(_workers(threads)) as ex:
        out = list(ex.map(lambda s: prob.run(vel, s), shots))
    return np.stack(out)


def misfit(a, b):
    """phi = 1/2 sum (a - b)^2 in FP64 (the paper's l2-norm misfit, Testing approach).

    Pinned by: zero at the truth, quadratic scaling, brute-force sums.
    """
    r = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return 0.5 * float(np.sum(r * r))


# Relative floor of the trace normalisation: a trace is divided by
# max(|trace|, w) with w = TRACE_FLOOR times the largest trace norm of the
# same shot's traces on the same side (modelled or observed), so that traces
# with no arrival (the scheme's precursor alone, many orders of magnitude
# below any arrival) are not raised to full weight, and each side stays
# invariant under a scale of all its traces.
TRACE_FLOOR = 1e-4


def trace_floor(x):
    """w of one shot's traces x[nt][nrec]."""
    x = np.asarray(x, dtype=np.float64)
    return TRACE_FLOOR * float(np.sqrt(np.sum(x * x, axis=0)).max())


def normalise_traces(d, w):
    """One shot's traces d[nt][nrec], each divided by max(its l2 norm, w); a
    trace for which that is zero stays zero."""
    d = np.asarray(d, dtype=np.float64)
    s = np.maximum(np.sqrt(np.sum(d * d, axis=0)), w)
    return np.divide(d, s, out=np.zeros_like(d), where=s > 0)


def misfit_normalised(a, b):
    """Trace-normalised misfit of modelled traces a against observed traces b,
    [nt][nrec] or [nshots][nt][nrec]: per shot, 1/2 sum over traces of
    |a/max(|a|, wa) - b/max(|b|, wb)|^2, wa and wb the floors of a and b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if not np.all(np.isfinite(a)):
        return math.inf
    if a.ndim == 3:
        return float(sum(misfit_normalised(a[s], b[s]) for s in range(a.shape[0])))
    return misfit(normalise_traces(a, trace_floor(a)), normalise_traces(b, trace_floor(b)))


def trace_misfit(prob, a, b):
    """The problem's misfit between modelled traces a and observed traces b."""
    return misfit_normalised(a, b) if prob.misfit == "trace_normalised" else misfit(a, b)


def fitness_batch(prob, nodes, d_obs, shots=None, threads=None):
    """Fitness of each particle: sum over shots of the misfit (Results section:
    a particle's fitness needs all 50 shots). nodes[P][D] FP64 (D node values),
    d_obs[nshots][nt][nrec]. Non-finite fitness maps to +inf.
    Returns (fitness[P], per-run misfit[P][len(shots)]).
    """
    nodes = np.atleast_2d(np.asarray(nodes, dtype=np.float64))
    shots = list(range(prob.nshots)) if shots is None else list(shots)
    vels = [pad_edge(prob.model(n), prob.nbl) for n in nodes]
    jobs = [(p, k, s) for p in range(len(nodes)) for k, s in enumerate(shots)]

    def one(job):
        p, k, s = job
        tr = prob.run(vels[p], s)
        return trace_misfit(prob, tr, d_obs[s])

    with ThreadPoolExecutor(_workers(threads)) as ex:
        vals = list(ex.map(one, jobs))
    per = np.array(vals, dtype=np.float64).reshape(len(nodes), len(shots))
    fit = per.sum(axis=1)
    fit[~np.isfinite(fit)] = np.inf
    return fit, per
