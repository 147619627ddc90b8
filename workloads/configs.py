"""The five benchmark workloads as plain geometry dictionaries.

Keys (all SI units: metres, seconds, m/s, Hz):
  nz, nx, dz, dx   physical grid (z down, slow index; x fast index); point (i, j)
                   sits at z = i*dz, x = j*dx, origin at the top-left corner.
  nbl              absorbing-layer thickness in grid points on every side.
  f0, tmax         Ricker peak frequency and record length.
  dt_frac, vmax    the time step is dt_frac times the leapfrog stability limit
                   at velocity vmax (both sides compute that limit themselves).
  src, rec         [n][2] (z, x) positions of shots and receivers.
  ncz, ncx         regular control-node grid (corners included).
  node_z, level_nodes, node_x
                   optional layered node grid instead (depth levels with
                   their own node x positions, metres; see layered_nodes).
  water_rows, v_water
                   optional water layer: the top physical rows are fixed.
  observed         optional {"f0", "f_pass", "f_stop"}: the observed data come
                   from a source of that peak frequency, low-passed.
  node_lo, node_hi [D] search box per node (row-major z-major, or level by level).
  damp_R           target reflection coefficient of the absorbing layer.
  model            recipe of the true model (generator name and seed).
  particles, particle_seed   swarm size and seed of the initial draw.

Config 2 is a list of three such dictionaries (three grid sizes in one batch).
"""
import numpy as np

from .models import two_layer, layered_faulted

CONFIG_NAMES = ("tiny", "realistic", "batched", "surrogate", "full", "mini", "irregular", "crime_free")


def _prior_box(nz, dz, ncz, ncx, v0=1500.0, v1=5500.0, lo_min=1400.0, hi_max=6000.0):
    """Search box centred on a 1-D prior increasing linearly with depth.

    Node row a sits at depth a*(nz-1)*dz/(ncz-1); its box is
    [max(lo_min, 0.7*v_prior), min(hi_max, 1.3*v_prior)].
    """
    zrow = np.arange(ncz) * (nz - 1) * dz / (ncz - 1)
    vprior = v0 + (v1 - v0) * zrow / ((nz - 1) * dz)
    lo = np.maximum(lo_min, 0.7 * vprior)
    hi = np.minimum(hi_max, 1.3 * vprior)
    return np.repeat(lo, ncx), np.repeat(hi, ncx)


def layered_nodes(nz, nx, dz, dx, water_rows, v0, v1, kz, kx):
    """Node layout built from a 1-D prior v(z) rising linearly from v0 at the
    water bottom to v1 at the grid bottom: the first level sits at the water
    bottom, each next level kz * v(z) deeper (the last one at the bottom of
    the grid), and level a holds evenly spaced nodes about kx * v(z_a) apart
    across the grid (at least 2), so the grid coarsens where the prior is
    faster. Returns (node_z, level_nodes, node_x, prior at each level)."""
    zw, zmax, xmax = water_rows * dz, (nz - 1) * dz, (nx - 1) * dx
    prior = lambda z: v0 + (v1 - v0) * (z - zw) / (zmax - zw)          # noqa: E731
    node_z = [zw]
    while node_z[-1] + kz * prior(node_z[-1]) < zmax - 0.5 * kz * prior(node_z[-1]):
        node_z.append(node_z[-1] + kz * prior(node_z[-1]))
    node_z.append(zmax)
    counts, xs = [], []
    for z in node_z:
        n = max(2, int(round(xmax / (kx * prior(z)))) + 1)
        counts.append(n)
        xs.append(np.linspace(0.0, xmax, n))
    return np.array(node_z), counts, np.concatenate(xs), np.array([prior(z) for z in node_z])


def _level_box(node_z, counts, prior, first=(0.8, 1.2), last=(0.7, 1.3), lo_min=1400.0, hi_max=6000.0):
    """Search box per node: the first and last levels span fractions of the
    prior velocity there; the bounds of the levels in between lie on the
    lines joining those of the first and last levels (linear in depth);
    everything is clipped to [lo_min, hi_max] (hi_max is the velocity the
    time step is chosen for)."""
    z0, z1 = node_z[0], node_z[-1]
    lo0, hi0 = first[0] * prior[0], first[1] * prior[0]
    lo1, hi1 = last[0] * prior[-1], last[1] * prior[-1]
    w = (node_z - z0) / (z1 - z0)
    lo = np.maximum(lo_min, lo0 + (lo1 - lo0) * w)
    hi = np.minimum(hi_max, hi0 + (hi1 - hi0) * w)
    return np.repeat(lo, counts), np.repeat(hi, counts)


def _surface_line(n, spacing):
    return [[0.0, k * spacing] for k in range(n)]


def _shots_even(nshots, nx, dx):
    """nshots sources on the surface at x = (s+1)*L/(nshots+1), snapped to the grid."""
    L = (nx - 1) * dx
    return [[0.0, round((s + 1) * L / (nshots + 1) / dx) * dx] for s in range(nshots)]


def _layered_geometry(nz, nx, h, nshots, rec_step, f0, tmax, ncz, ncx, seed, pseed, npart):
    lo, hi = _prior_box(nz, h, ncz, ncx)
    nrec = (nx - 1) * h // rec_step + 1
    return {
        "nz": nz, "nx": nx, "dz": float(h), "dx": float(h), "nbl": 40,
        "f0": float(f0), "tmax": float(tmax), "dt_frac": 0.4, "vmax": 6000.0,
        "src": _shots_even(nshots, nx, float(h)),
        "rec": _surface_line(int(nrec), float(rec_step)),
        "ncz": ncz, "ncx": ncx, "node_lo": lo, "node_hi": hi,
        "damp_R": 1e-3,
        "model": {"kind": "layered_faulted", "seed": seed},
        "particles": npart, "particle_seed": pseed,
    }


def config(name):
    """Return the geometry dictionary (or list of them) of a named workload."""
    if name in ("tiny", 0):
        nz = nx = 101
        return {
            "nz": nz, "nx": nx, "dz": 10.0, "dx": 10.0, "nbl": 40,
            "f0": 10.0, "tmax": 1.0, "dt_frac": 0.4, "vmax": 2700.0,
            "src": [[0.0, 500.0]],
            "rec": _surface_line(101, 10.0),
            "ncz": 2, "ncx": 3,
            "node_lo": np.full(6, 1400.0), "node_hi": np.full(6, 2700.0),
            "damp_R": 1e-3,
            "model": {"kind": "two_layer", "seed": 1, "v_top": 1500.0, "v_bottom": 2500.0},
            "particles": 8, "particle_seed": 2,
        }
    if name in ("realistic", 1, "surrogate", 3):
        g = _layered_geometry(301, 921, 10, 16, 20, 5.0, 3.0, 5, 12, seed=3, pseed=4, npart=32)
        if name in ("surrogate", 3):
            g["particles"] = 64
            g["candidates_per_particle"] = 16
        return g
    if name in ("batched", 2):
        out = []
        for (nz, nx), seed in zip(((201, 601), (301, 921), (401, 1201)), (5, 6, 7)):
            out.append(_layered_geometry(nz, nx, 10, 16, 20, 5.0, 3.0, 5, 12,
                                         seed=seed, pseed=10, npart=64))
        return out
    if name in ("full", 4):
        return _layered_geometry(601, 1841, 5, 32, 10, 6.0, 4.0, 8, 20, seed=8, pseed=9, npart=128)
    if name == "crime_free":
        # the realistic geometry fitted the way the paper fits its data: the
        # modelled source has a 6 Hz maximum frequency (peak 3 Hz), the
        # observed data come from a 17 Hz source (peak 8.5 Hz) low-passed
        # between 5 and 6 Hz, so no model reproduces them exactly
        g = _layered_geometry(301, 921, 10, 16, 20, 3.0, 3.0, 5, 12, seed=3, pseed=4, npart=32)
        g["observed"] = {"f0": 8.5, "f_pass": 5.0, "f_stop": 6.0}
        return g
    if name == "irregular":
        # the realistic acquisition with the paper's kind of parameterisation:
        # a layered node grid from a 1-D prior (1500 -> 5500 m/s), a water
        # layer of 4 rows at 1500 m/s, and depth-dependent search ranges
        g = _layered_geometry(301, 921, 10, 16, 20, 5.0, 3.0, 5, 12, seed=3, pseed=4, npart=32)
        del g["ncz"], g["ncx"]
        g["water_rows"], g["v_water"] = 4, 1500.0
        node_z, counts, node_x, prior = layered_nodes(301, 921, 10.0, 10.0, 4, 1500.0, 5500.0, 0.12, 0.6)
        g["node_z"], g["level_nodes"], g["node_x"] = node_z, counts, node_x
        g["node_lo"], g["node_hi"] = _level_box(node_z, counts, prior)
        return g
    if name == "mini":
        # a reduced realistic search used to compare plain and screened swarms
        # quickly: 1 km x 3 km at 10 m, 4 shots, 151 receivers, 4 Hz, 1.5 s,
        # 3 x 6 nodes, 32 particles; true model layered and faulted, 1500-2800 m/s
        g = _layered_geometry(101, 301, 10, 4, 20, 4.0, 1.5, 3, 6, seed=3, pseed=1, npart=32)
        g["src"] = [[0.0, x] for x in (500.0, 1200.0, 1800.0, 2500.0)]
        g["model"] = {"kind": "layered_faulted", "seed": 3, "v_bottom": 2800.0}
        zrow = np.arange(3) * 1000.0 / 2
        vprior = 1500.0 + 4000.0 * zrow / 3000.0
        g["node_lo"] = np.repeat(np.maximum(1400.0, 0.7 * vprior), 6)
        g["node_hi"] = np.repeat(np.minimum(6000.0, 1.3 * vprior), 6)
        return g
    raise KeyError(name)


def true_model(geom):
    """Generate the seeded true velocity model vp[nz][nx] (float64) of a geometry
    (with its water layer, if it has one)."""
    m = geom["model"]
    if m["kind"] == "two_layer":
        vp, _ = two_layer(geom["nz"], geom["nx"], geom["dz"], geom["dx"],
                          m["v_top"], m["v_bottom"], m["seed"])
    elif m["kind"] == "layered_faulted":
        vp = layered_faulted(geom["nz"], geom["nx"], geom["dz"], geom["dx"], m["seed"],
                             v_bottom=m.get("v_bottom", 5500.0))
    else:
        raise KeyError(m["kind"])
    w = int(geom.get("water_rows", 0))
    if w:
        vp[:w, :] = geom["v_water"]
    return vp
