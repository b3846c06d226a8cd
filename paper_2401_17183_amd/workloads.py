"""Seeded synthetic workloads: body-fitted mesh coordinates and initial fields.

This module only generates inputs (node positions from analytic mappings and
seeded random initial velocities).  It contains none of the method's
arithmetic and is shared by the HIP path, the tests and the oracle-based
checks, which is its only purpose.

Every workload is a plain dict:
  lattice   "D2Q9" | "D3Q19"
  n         (n_1, .., n_d) real cells per index axis (q^1 fastest in memory)
  coords    float64 (m_d, .., m_1, d); m_i = n_i + 4 on non-periodic axes
  faces     per axis (low, high) in {PERIODIC, WALL, FARFIELD}
  wrap      per axis translation vector (periodic axes)
  dx        representative spacing (the Delta x of the tangent-vector formula)
  tau, body_force, rho_inf, u_inf, and optional init fields rho (*n), u (d, *n)
"""
import numpy as np

PERIODIC, WALL, FARFIELD = 0, 1, 2
NGHOST = 2
SEED = 2401


# lattices whose links span three cells: four ghost node layers per wall face,
# and their lattice temperature (the others: two layers, T0 = 1/3)
LONG_LINK = {"D2Q21": 2.0 / 3.0, "D3Q39": 2.0 / 3.0}


def ghost_layers(lattice):
    return 4 if lattice in LONG_LINK else NGHOST


def _cell_eta(n, lo=-1.0, hi=1.0, ghost=NGHOST):
    """Cell-centred parameter values, `ghost` layers each side."""
    j = np.arange(-ghost, n + ghost)
    return lo + (j + 0.5) * (hi - lo) / n


def _central_min(y, ghost=NGHOST):
    """Smallest central spacing (y_{j+1} - y_{j-1}) / 2 over real nodes."""
    yr = y[ghost - 1: len(y) - ghost + 1]
    return float(np.min((yr[2:] - yr[:-2]) / 2.0))


def tanh_channel_2d(n1=64, n2=32, strength=2.0, tau=0.8, G=1e-6, lattice="D2Q9", dx_ratio=np.sqrt(3.0)):
    """Plane channel, periodic x, walls at y = +-1, y = tanh(s eta)/tanh(s).

    dx = dx_ratio * (smallest central wall-normal spacing), streamwise spacing
    dx.  lattice D2Q21 carries four ghost node layers per wall face.
    """
    ng = ghost_layers(lattice)
    eta = _cell_eta(n2, ghost=ng)
    y = np.tanh(strength * eta) / np.tanh(strength)
    dx = dx_ratio * _central_min(y, ng)
    x = np.arange(n1) * dx
    X = np.empty((len(y), n1, 2))
    X[..., 0] = x[None, :]
    X[..., 1] = y[:, None]
    return {
        "name": f"{lattice} tanh({strength}) channel {n1}x{n2}",
        "lattice": lattice, "ghost": ng, "n": (n1, n2), "coords": X,
        "faces": [(PERIODIC, PERIODIC), (WALL, WALL)],
        "wrap": [(n1 * dx, 0.0), (0.0, 0.0)], "dx": dx,
        "tau": tau, "body_force": (G, 0.0), "half_height": 1.0 / dx,
    }


def poiseuille_fields(w):
    """Analytic plane Poiseuille profile u = G (H^2 - Y^2) / (2 nu) in lattice
    units (Y, H in units of dx), rho = 1; used as the initial state."""
    n1, n2 = w["n"]
    nu = (w["tau"] - 0.5) * LONG_LINK.get(w["lattice"], 1.0 / 3.0)
    ng = w.get("ghost", NGHOST)
    y = w["coords"][ng:ng + n2, 0, 1] / w["dx"]
    H = w["half_height"]
    G = w["body_force"][0]
    ux = G * (H * H - y * y) / (2.0 * nu)
    u = np.zeros((2, n2, n1))
    u[0] = ux[:, None]
    return np.ones((n2, n1)), u


def tanh_channel_3d(n1=256, n2=128, n3=128, strength=2.5, tau=0.52, G=1e-6,
                    noise=1e-3, seed=SEED, lattice="D3Q19", dx_ratio=np.sqrt(3.0)):
    """Channel: x, z periodic, walls at y = +-1, y = tanh(s eta)/tanh(s);
    initial rho = 1, u ~ U(-noise, noise) per component (seeded);
    dx = dx_ratio * (smallest central wall-normal spacing)."""
    ng = ghost_layers(lattice)
    eta = _cell_eta(n2, ghost=ng)
    y = np.tanh(strength * eta) / np.tanh(strength)
    dx = dx_ratio * _central_min(y, ng)
    X = np.empty((n3, len(y), n1, 3))
    X[..., 0] = (np.arange(n1) * dx)[None, None, :]
    X[..., 1] = y[None, :, None]
    X[..., 2] = (np.arange(n3) * dx)[:, None, None]
    rng = np.random.default_rng(seed)
    u = rng.uniform(-noise, noise, size=(3, n3, n2, n1))
    return {
        "name": f"{lattice} tanh({strength}) channel {n1}x{n2}x{n3}",
        "lattice": lattice, "ghost": ng, "n": (n1, n2, n3), "coords": X,
        "faces": [(PERIODIC, PERIODIC), (WALL, WALL), (PERIODIC, PERIODIC)],
        "wrap": [(n1 * dx, 0, 0), (0, 0, 0), (0, 0, n3 * dx)], "dx": dx,
        "tau": tau, "body_force": (G, 0.0, 0.0),
        "rho": np.ones((n3, n2, n1)), "u": u,
    }


def ogrid_3d(nr=256, nth=512, nz=64, rmax=20.0, u_inf=0.05, Re=100.0, dx_factor=1.0):
    """O-grid around a unit cylinder: r = rmax^(k/(nr-1)) (log spaced), theta
    periodic, z periodic with spacing dx; wall at r = 1, far field at r = rmax.
    dx = dx_factor * (radial spacing at r = 1); nu from Re = u_inf * (2 / dx) / nu."""
    k = np.arange(-NGHOST, nr + NGHOST)
    r = rmax ** (k / (nr - 1.0))
    dx = dx_factor * float(r[NGHOST + 1] - r[NGHOST])
    th = 2.0 * np.pi * np.arange(nth) / nth
    z = np.arange(nz) * dx
    X = np.empty((nz, nth, len(r), 3))
    X[..., 0] = (r[None, None, :] * np.cos(th)[None, :, None])
    X[..., 1] = (r[None, None, :] * np.sin(th)[None, :, None])
    X[..., 2] = z[:, None, None]
    nu = u_inf * (2.0 / dx) / Re
    tau = 3.0 * nu + 0.5
    return {
        "name": f"D3Q19 O-grid {nr}x{nth}x{nz}",
        "lattice": "D3Q19", "n": (nr, nth, nz), "coords": X,
        "faces": [(WALL, FARFIELD), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)],
        "wrap": [(0, 0, 0), (0, 0, 0), (0, 0, nz * dx)], "dx": dx,
        "tau": tau, "body_force": (0.0, 0.0, 0.0),
        "rho_inf": 1.0, "u_inf": (u_inf, 0.0, 0.0),
    }


def _stretch01(eta, s):
    """Map [0,1] -> [0,1], clustering at both ends with centre/wall spacing ~ s."""
    if s <= 1.0 + 1e-12:
        return eta
    sig = np.arccosh(np.sqrt(s))
    return 0.5 * (1.0 + np.tanh(sig * (2.0 * eta - 1.0)) / np.tanh(sig))


def bump_channel_2d(n1, n2, bump, stretch, tau, G=1e-6, H=1.0, max_slope=0.15):
    """Periodic-x channel with a lower wall bump y_b = bump * sin^8(pi x / L)
    and a flat upper wall at H; wall-normal tanh clustering of ratio ~stretch.

    dx = sqrt(2) * the smallest wall-normal spacing anywhere (the bump crest
    squeezes the first cell by (H - bump) / H), streamwise spacing dx, L = n1 dx.
    The bump height is capped so that the steepest wall slope,
    (8 pi / L) * bump * max(sin^7 cos) = 5.59 bump / L, stays at most max_slope:
    skewed, squeezed cells otherwise leave the window of metrics for which the
    rest populations stay positive."""
    eta = (np.arange(-NGHOST, n2 + NGHOST) + 0.5) / n2
    prof = _stretch01(eta, stretch)
    hmin = _central_min(prof * H)
    peak = 8.0 * np.pi * (7.0 / 8.0) ** 3.5 * np.sqrt(1.0 / 8.0)
    bump = min(bump, max_slope * n1 * np.sqrt(2.0) * hmin * (1.0 - bump / H) / peak)
    dx = np.sqrt(2.0) * hmin * (1.0 - bump / H)
    L = n1 * dx
    x = np.arange(n1) * dx
    yb = bump * np.sin(np.pi * x / L) ** 8
    X = np.empty((len(eta), n1, 2))
    X[..., 0] = x[None, :]
    X[..., 1] = yb[None, :] + (H - yb[None, :]) * prof[:, None]
    return {
        "name": f"D2Q9 bump channel {n1}x{n2}",
        "lattice": "D2Q9", "n": (n1, n2), "coords": X,
        "faces": [(PERIODIC, PERIODIC), (WALL, WALL)],
        "wrap": [(L, 0.0), (0.0, 0.0)], "dx": dx,
        "tau": tau, "body_force": (G, 0.0),
        "bump": bump, "stretch": stretch, "H": H,
    }


def batch_meshes(count=256, seed=SEED, max_slope=0.15):
    """The uneven batch: n1 ~ U{32..256}, n2 ~ U{16..128}, bump ~ U[0, 0.3] H
    (then capped by the wall-slope limit max_slope of bump_channel_2d; None:
    uncapped), stretch ~ U[1, 3], tau ~ U[0.55, 1.0]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n1 = int(rng.integers(32, 257))
        n2 = int(rng.integers(16, 129))
        bump = float(rng.uniform(0.0, 0.3))
        s = float(rng.uniform(1.0, 3.0))
        tau = float(rng.uniform(0.55, 1.0))
        out.append(bump_channel_2d(n1, n2, bump, s, tau, max_slope=np.inf if max_slope is None else max_slope))
    return out


def channel_vortex_fields(w, amp=0.02):
    """A smooth initial state for a 2D channel member: rho = 1 and, with
    xi = (q^1 + 1/2) / n_1, eta = (q^2 + 1/2) / n_2,
    u_x = amp sin(pi eta) (1 + 0.3 sin(2 pi xi)), u_y = (amp / 2) sin(2 pi eta) cos(2 pi xi).
    Returns rho (n_2, n_1) and u (2, n_2, n_1)."""
    n1, n2 = w["n"]
    xi = (np.arange(n1) + 0.5) / n1
    eta = (np.arange(n2) + 0.5) / n2
    u = np.empty((2, n2, n1))
    u[0] = amp * np.sin(np.pi * eta)[:, None] * (1.0 + 0.3 * np.sin(2 * np.pi * xi))[None, :]
    u[1] = 0.5 * amp * np.sin(2 * np.pi * eta)[:, None] * np.cos(2 * np.pi * xi)[None, :]
    return np.ones((n2, n1)), u


def surrogate_meshes(count, seed=SEED, n1=128, n2=64, u_bulk=0.05, re_range=(10.0, 100.0)):
    """Bump channels at n1 x n2 with bump ~ U[0, 0.3] H (slope-capped as in
    bump_channel_2d), stretch ~ U[1, 3], Re ~ U[re_range].  The bulk velocity is
    held at u_bulk (Mach ~0.1 at the centreline) and the viscosity follows from
    Re = u_bulk H / nu with H the channel height in units of dx:
    nu = u_bulk H / Re, tau = 1/2 + 3 nu, and G = 12 nu u_bulk / H^2 from the
    flat-channel relation u_bulk = G H^2 / (12 nu)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        bump = float(rng.uniform(0.0, 0.3))
        s = float(rng.uniform(1.0, 3.0))
        Re = float(rng.uniform(*re_range))
        w = bump_channel_2d(n1, n2, bump, s, 0.8)
        Hl = w["H"] / w["dx"]
        nu = u_bulk * Hl / Re
        w["tau"] = 0.5 + 3.0 * nu
        w["body_force"] = (12.0 * nu * u_bulk / Hl ** 2, 0.0)
        w["Re"] = Re
        w["u_bulk"] = u_bulk
        out.append(w)
    return out


def affine_mesh(lattice, n, Amat, origin=None, periodic=True):
    """x = origin + Amat q (uniform sheared/stretched lattice); periodic in all
    axes (or walls on axis 2 when periodic is False)."""
    d = len(n)
    Amat = np.asarray(Amat, dtype=np.float64)
    origin = np.zeros(d) if origin is None else np.asarray(origin, dtype=np.float64)
    axes = []
    faces = []
    wrap = []
    for i in range(d):
        per = periodic or i != 1
        q = np.arange(n[i]) if per else np.arange(-NGHOST, n[i] + NGHOST)
        axes.append(q.astype(np.float64))
        faces.append((PERIODIC, PERIODIC) if per else (WALL, WALL))
        wrap.append(tuple(Amat[:, i] * n[i]) if per else tuple([0.0] * d))
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    qs = [grids[d - 1 - i] for i in range(d)]
    X = np.zeros(grids[0].shape + (d,))
    for k in range(d):
        X[..., k] = origin[k] + sum(Amat[k, i] * qs[i] for i in range(d))
    return {"name": "affine", "lattice": lattice, "n": tuple(n), "coords": X,
            "faces": faces, "wrap": wrap, "dx": 1.0, "tau": 0.8,
            "body_force": tuple([0.0] * d)}


def wavy_periodic(lattice, n, amp=0.15, seed=SEED, dx=1.0):
    """Fully periodic mesh with smooth sinusoidal node displacements:
    x^k = q^k + amp * sum of sines of the other index coordinates; a
    curvilinear mesh with no boundary, used for the conservation checks."""
    d = len(n)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=(d, d))
    axes = [np.arange(n[i], dtype=np.float64) for i in range(d)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    qs = [grids[d - 1 - i] for i in range(d)]
    X = np.zeros(grids[0].shape + (d,))
    for k in range(d):
        X[..., k] = qs[k]
        for i in range(d):
            if i != k:
                X[..., k] += amp * np.sin(2 * np.pi * qs[i] / n[i] + ph[k, i])
    X *= dx
    wrap = [tuple(dx * n[i] * (np.arange(d) == i)) for i in range(d)]
    return {"name": f"{lattice} wavy periodic {n}", "lattice": lattice, "n": tuple(n),
            "coords": X, "faces": [(PERIODIC, PERIODIC)] * d, "wrap": wrap, "dx": dx,
            "tau": 0.8, "body_force": tuple([0.0] * d)}


def wavy_channel_3d(n1=16, n2=12, n3=8, amp=0.1, strength=1.0, tau=0.7, G=1e-5, seed=SEED):
    """Small 3-D curvilinear channel: tanh wall-normal clustering plus a smooth
    wall-parallel waviness of every node coordinate; periodic x, z; walls on y.
    dx = 1.1 * smallest central wall-normal spacing keeps the rest equilibrium
    positive.  Exercises every A^i_a."""
    eta = _cell_eta(n2)
    yb = np.tanh(strength * eta) / np.tanh(strength)
    dx = 1.1 * _central_min(yb)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=4)
    i = np.arange(n1, dtype=np.float64)[None, None, :]
    k = np.arange(n3, dtype=np.float64)[:, None, None]
    y = yb[None, :, None]
    X = np.empty((n3, len(eta), n1, 3))
    X[..., 0] = i * dx + amp * dx * np.sin(2 * np.pi * k / n3 + ph[0]) * (1 - y * y)
    X[..., 1] = y + amp * dx * np.sin(2 * np.pi * i / n1 + ph[1]) * (1 - y * y) \
        + 0.5 * amp * dx * np.sin(2 * np.pi * k / n3 + ph[2]) * (1 - y * y)
    X[..., 2] = k * dx + amp * dx * np.sin(2 * np.pi * i / n1 + ph[3]) * (1 - y * y)
    rng2 = np.random.default_rng(seed + 1)
    u = rng2.uniform(-1e-3, 1e-3, size=(3, n3, n2, n1))
    return {"name": f"D3Q19 wavy channel {n1}x{n2}x{n3}", "lattice": "D3Q19",
            "n": (n1, n2, n3), "coords": X,
            "faces": [(PERIODIC, PERIODIC), (WALL, WALL), (PERIODIC, PERIODIC)],
            "wrap": [(n1 * dx, 0, 0), (0, 0, 0), (0, 0, n3 * dx)], "dx": dx,
            "tau": tau, "body_force": (G, 0.0, 0.0), "rho": np.ones((n3, n2, n1)), "u": u}


def moving_coords(w, t, breathe=0.0, omega=0.0, velocity=None, period=40.0):
    """Node positions and periodic translations of a periodic workload w at
    integer time t for a mesh in motion: the displacement of w's nodes from
    the uniform lattice (x - dx q) scaled by 1 + breathe sin(2 pi t / period)
    (a deforming mesh), the whole mesh turned by the angle omega t about the
    last axis (a rigid rotation in the (x, y) plane) and shifted by
    velocity * t (a rigid translation).  Returns (coords (t), wrap (t));
    t = 0 gives w's own mesh when breathe only scales."""
    d = len(w["n"])
    X = np.array(w["coords"], dtype=np.float64)
    dx = w["dx"]
    axes = [np.arange(w["n"][i], dtype=np.float64) for i in range(d)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    base = np.stack([grids[d - 1 - i] * dx for i in range(d)], axis=-1)
    X = base + (X - base) * (1.0 + breathe * np.sin(2.0 * np.pi * t / period))
    wrap = np.array([np.asarray(v, dtype=np.float64)[:d] for v in w["wrap"]])
    th = omega * t
    R = np.eye(d)
    R[0, 0], R[0, 1], R[1, 0], R[1, 1] = np.cos(th), -np.sin(th), np.sin(th), np.cos(th)
    X = X @ R.T
    wrap = wrap @ R.T
    if velocity is not None:
        X = X + np.asarray(velocity, dtype=np.float64)[:d] * t
    return X, wrap
