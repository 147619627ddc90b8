"""Seeded synthetic velocity models and particle draws.

The paper's test model is a cropped Marmousi section (Testing approach section),
which is not available here. These generators stand in for it with the same
extent and velocity range: water-like velocity at the top, increasing with
depth to about 5.5 km/s, folded interfaces and normal faults, plus a small
smooth random perturbation.
"""
import numpy as np


def two_layer(nz, nx, dz, dx, v_top, v_bottom, seed, zmin=400.0, zmax=600.0):
    """Two flat layers; the interface depth is drawn U(zmin, zmax) metres.

    Returns (vp[nz][nx] float64, interface_depth_m).
    """
    rng = np.random.default_rng(seed)
    zi = float(rng.uniform(zmin, zmax))
    z = np.arange(nz, dtype=np.float64) * dz
    vp = np.where(z[:, None] < zi, v_top, v_bottom) * np.ones((1, nx))
    return vp.astype(np.float64), zi


def layered_faulted(nz, nx, dz, dx, seed, nlayers=8, v_top=1500.0, v_bottom=5500.0,
                    nfaults=3, dip_deg=60.0, throw=(50.0, 200.0), fold_amp=(50.0, 200.0),
                    fold_len=(2000.0, 8000.0), perturb=0.05, sigma_pts=20.0):
    """Layered model with folded interfaces, normal faults and a smooth perturbation.

    * ``nlayers`` layers separated by ``nlayers-1`` interfaces. Interface k has a
      base depth near (k+1)/nlayers of the section depth (jitter of +-30 % of the
      spacing) and a sinusoidal fold of amplitude U(fold_amp) and wavelength
      U(fold_len) with a random phase.
    * Layer k has velocity v_top + (v_bottom - v_top) * k / (nlayers - 1).
    * ``nfaults`` planar normal faults with the given dip, surface trace
      x ~ U(0.15, 0.85) of the section width, random dip direction, throw
      U(throw). Points on the hanging wall see the layering displaced down by
      the throw; faults are applied in sequence.
    * The result is multiplied by (1 + perturb * g), where g is white noise
      smoothed by a Gaussian of ``sigma_pts`` grid points and scaled to
      max |g| = 1.

    Returns vp[nz][nx] float64.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    Z = (nz - 1) * dz
    X = (nx - 1) * dx
    z = np.arange(nz, dtype=np.float64)[:, None] * dz
    x = np.arange(nx, dtype=np.float64)[None, :] * dx

    spacing = Z / nlayers
    base = (np.arange(1, nlayers) * spacing
            + rng.uniform(-0.3, 0.3, nlayers - 1) * spacing)
    amp = rng.uniform(*fold_amp, nlayers - 1)
    lam = rng.uniform(*fold_len, nlayers - 1)
    phase = rng.uniform(0.0, 2.0 * np.pi, nlayers - 1)

    xf = rng.uniform(0.15, 0.85, nfaults) * X
    fdir = rng.choice([-1.0, 1.0], nfaults)
    fthrow = rng.uniform(*throw, nfaults)
    tan_dip = np.tan(np.deg2rad(dip_deg))

    zeff = np.broadcast_to(z, (nz, nx)).copy()
    for f in range(nfaults):
        side = (x - xf[f]) * fdir[f] - z / tan_dip
        zeff = np.where(side > 0.0, zeff - fthrow[f], zeff)

    layer = np.zeros((nz, nx), dtype=np.int64)
    for k in range(nlayers - 1):
        zk = base[k] + amp[k] * np.sin(2.0 * np.pi * x / lam[k] + phase[k])
        layer += (zeff >= zk).astype(np.int64)
    vlayer = v_top + (v_bottom - v_top) * np.arange(nlayers) / (nlayers - 1)
    vp = vlayer[layer]

    g = gaussian_filter(rng.standard_normal((nz, nx)), sigma=sigma_pts, mode="nearest")
    g /= np.max(np.abs(g))
    return (vp * (1.0 + perturb * g)).astype(np.float64)


def uniform_particles(n, lo, hi, seed):
    """n particles drawn uniformly in the box [lo, hi] (per-dimension arrays)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((n, lo.size))


def mlp_init(sizes, seed):
    """Seeded initial weights of a fully connected network: per layer
    W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) of shape [fan_out][fan_in], then
    b ~ the same range. Returns [(W, b), ...] in float64."""
    rng = np.random.default_rng(seed)
    out = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        s = 1.0 / np.sqrt(fin)
        out.append((rng.uniform(-s, s, (fout, fin)), rng.uniform(-s, s, fout)))
    return out
