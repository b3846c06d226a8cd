"""Geometry of a body-fitted mesh (Sec. 2.1).

Index conventions.  A mesh has d index axes q = (q^1, .., q^d) with n_i cells on
axis i.  NumPy arrays over cells are stored with the LAST axis = q^1 (so a C
order flatten gives cell = q^1 + n_1 (q^2 + n_2 q^3)).  Vector-valued fields
carry their component index first.

Boundary readings (the paper leaves boundaries out of its scope):
* every non-periodic face carries two ghost node layers in the coordinate
  input, so that g_i exists on the first ghost layer and the contracted
  coefficient A (below) exists on every link of every real cell;
* lattices with links longer than one cell (D2Q21, D3Q39, longest link s = 3
  cells) need g_i s cells beyond every real cell: a non-periodic face then
  carries s + 1 ghost node layers (ghost_layers()).  Such a lattice takes walls
  on at most one axis (no corners) and no far-field faces;
* a periodic axis i wraps the index and translates positions by a constant
  vector L_i: x(q + n_i e_i) = x(q) + L_i.

Quantities and the equations they follow:
* D_{+-i}(q) = x(q +- e_i) - x(q)                                  eq. (distance)
* beta_i = (|D_i| + |D_-i|) / |D_i - D_-i|,
  g_i = beta_i (D_i - D_-i) / (2 dx)                               eq. (tangent)
* J = (g_1 x g_2) . g_3  (2-D: the scalar cross product)          eq. (jacobian)
* g^1 = g_2 x g_3 / J and cyclic (2-D: the planar analogue)       eq. (covectors)
* g^{ij} = g^i . g^j                                               eq. (inverse)
* e_a(q) = c_a^i g_i(q)                                            eq. (lattice)
* Theta^i_j(q + c_a, q) = [g_j(q + c_a) - g_j(q)] . g^i(q)          eq. (gamma)

The inertial force only ever uses Theta contracted with the link velocity,
A^i_a(q) = sum_j c_a^j Theta^i_j(q + c_a, q) = [e_a(q + c_a) - e_a(q)] . g^i(q),
and, because c_{opp(a)} = -c_a, sum_j c_a^j Theta^i_j(q - c_a, q) = -A^i_{opp(a)}(q).

Pinned by: g_i . g^j = delta, g^{ij} = [g_ij]^-1, det g_ij = J^2 (eq. (determinant)),
beta = 1 on collinear nodes, parity of g_i, Theta = 0 on a uniform lattice and on
any affine mesh, and second-order convergence of Theta to the Christoffel
symbols of an analytic mapping (the continuum limit in Sec. 3) and of
Gamma^i_{ij} to d_j ln J (App. C) -- tests/test_oracle_geometry.py.
"""
import numpy as np

PERIODIC, WALL, FARFIELD = 0, 1, 2
NGHOST = 2


def ghost_layers(lat):
    """Ghost node layers a non-periodic face carries: one more than the
    longest link (2 for D2Q9 / D3Q19, 4 for D2Q21 / D3Q39)."""
    return lat.speed + 1


class MeshError(ValueError):
    """Degenerate mesh: beta undefined (D_i = D_-i) or J <= 0."""


class Mesh:
    """A body-fitted mesh.

    n      : tuple (n_1, .., n_d) of real cells per index axis
    coords : float64 array (m_d, .., m_1, d); m_i = n_i + 2 ghost_layers on
             non-periodic axes, m_i = n_i on periodic axes
    faces  : per axis (low, high) kinds, PERIODIC on both faces or on neither
    wrap   : per axis translation L_i (length-d vector; ignored unless periodic)
    dx     : the representative spacing of eq. (tangent)
    """

    def __init__(self, lattice, n, coords, faces, wrap, dx):
        self.lat = lattice
        self.d = lattice.d
        self.n = tuple(int(v) for v in n)
        assert len(self.n) == self.d
        self.faces = [tuple(f) for f in faces]
        for lo, hi in self.faces:
            if (lo == PERIODIC) != (hi == PERIODIC):
                raise MeshError("an axis must be periodic on both faces or on neither")
        self.wrap = np.zeros((self.d, self.d))
        for i in range(self.d):
            self.wrap[i] = np.asarray(wrap[i], dtype=np.float64)[: self.d]
        self.dx = float(dx)
        if self.lat.speed > 1:
            walls = [i for i, f in enumerate(self.faces) if f[0] != PERIODIC]
            if any(FARFIELD in f for f in self.faces) or len(walls) > 1:
                raise MeshError(f"{self.lat.name} takes walls on at most one axis and no far field")
            if any(n < self.lat.speed for n in self.n):
                raise MeshError(f"{self.lat.name} needs at least {self.lat.speed} cells per axis")
        self.coords = np.asarray(coords, dtype=np.float64)
        want = tuple(reversed([self.m(i) for i in range(self.d)])) + (self.d,)
        if self.coords.shape != want:
            raise MeshError(f"coords shape {self.coords.shape} != {want}")

    def periodic(self, i):
        return self.faces[i][0] == PERIODIC

    def m(self, i):
        return self.n[i] if self.periodic(i) else self.n[i] + 2 * ghost_layers(self.lat)

    @property
    def shape(self):
        """NumPy shape of a real-cell field."""
        return tuple(reversed(self.n))

    @property
    def ncells(self):
        return int(np.prod(self.n))


def padded_coords(mesh, layers=None):
    """x(q) for q^i in [-layers, n_i + layers) on every axis.

    Non-periodic axes read the supplied ghost layers; periodic axes wrap the
    index and add the translation L_i per wrap.  layers defaults to the ghost
    layers of the lattice.
    """
    if layers is None:
        layers = ghost_layers(mesh.lat)
    d = mesh.d
    ng = ghost_layers(mesh.lat)
    idx = []
    shifts = []
    for i in range(d):
        q = np.arange(-layers, mesh.n[i] + layers)
        if mesh.periodic(i):
            idx.append(np.mod(q, mesh.n[i]))
            shifts.append(np.floor_divide(q, mesh.n[i]).astype(np.float64))
        else:
            if layers > ng:
                raise MeshError("not enough ghost layers")
            idx.append(q + ng)
            shifts.append(np.zeros(q.shape))
    # numpy axis order is (q^d, .., q^1)
    P = mesh.coords[np.ix_(*reversed(idx))].copy()
    for i in range(d):
        shape = [1] * d
        shape[d - 1 - i] = -1
        P += shifts[i].reshape(shape)[..., None] * mesh.wrap[i]
    return P


def _view(arr, lead, offset, box_layers, layers_out):
    """Sub-box of a field given on q in [-box_layers, n + box_layers): the part
    on q + offset for q in [-layers_out, n + layers_out)."""
    d = len(offset)
    sl = [slice(None)] * lead
    full = arr.shape[lead:]
    for ax in range(d):
        i = d - 1 - ax
        lo = box_layers - layers_out + offset[i]
        hi = full[ax] - box_layers + layers_out + offset[i]
        sl.append(slice(lo, hi))
    return arr[tuple(sl)]


def _cross2(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _cross3(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def box_layers(mesh):
    """Layers around the real cells on which basis() gives g_i: the longest
    link of the lattice (1 for D2Q9 / D3Q19)."""
    return mesh.lat.speed


def basis(mesh):
    """g_i, J, g^i, g^{ij} on real cells plus box_layers(mesh) layers around
    them (one for D2Q9 / D3Q19).

    Returns dict with arrays on the box q in [-s, n + s), s = box_layers(mesh):
      g    (d, d, *box): g[i] is the tangent vector g_i (eq. (tangent))
      J    (*box)                                   (eq. (jacobian))
      gco  (d, d, *box): gco[i] is the co-tangent g^i (eq. (covectors))
      gup  (d, d, *box): g^{ij}                      (eq. (inverse))
      beta (d, *box)
    Raises MeshError when beta is undefined or J <= 0 anywhere on the box.
    """
    d = mesh.d
    L = box_layers(mesh)
    P = np.moveaxis(padded_coords(mesh, L + 1), -1, 0)  # (d, *box of L + 1 layers)
    g = []
    beta = []
    for i in range(d):
        e = [0] * d
        e[i] = 1
        me = [0] * d
        me[i] = -1
        x0 = _view(P, 1, [0] * d, L + 1, L)
        Dp = _view(P, 1, e, L + 1, L) - x0        # D_{+i}
        Dm = _view(P, 1, me, L + 1, L) - x0       # D_{-i}
        diff = Dp - Dm
        nd = np.sqrt(np.sum(diff * diff, axis=0))
        if np.any(nd == 0.0):
            raise MeshError(f"beta_{i + 1} undefined: D_+ == D_- somewhere")
        b = (np.sqrt(np.sum(Dp * Dp, axis=0)) + np.sqrt(np.sum(Dm * Dm, axis=0))) / nd
        beta.append(b)
        g.append(b * diff / (2.0 * mesh.dx))
    g = np.stack(g)          # (i, component, *box)
    beta = np.stack(beta)
    if d == 2:
        J = _cross2(g[0], g[1])
    else:
        J = np.sum(_cross3(g[0], g[1]) * g[2], axis=0)
    if np.any(~(J > 0.0)):
        raise MeshError("J <= 0 somewhere (reorder the axes for a positive handedness)")
    if d == 2:
        gco = np.stack([np.stack([g[1][1], -g[1][0]]) / J,
                        np.stack([-g[0][1], g[0][0]]) / J])
    else:
        gco = np.stack([_cross3(g[1], g[2]) / J,
                        _cross3(g[2], g[0]) / J,
                        _cross3(g[0], g[1]) / J])
    gup = np.einsum("ik...,jk...->ij...", gco, gco)
    return {"g": g, "J": J, "gco": gco, "gup": gup, "beta": beta}


def link_coefficients(mesh, bas):
    """A^i_a(q) = [e_a(q + c_a) - e_a(q)] . g^i(q) on real cells.

    Shape (Q, d, *n).  This is eq. (gamma) contracted with c_a^j; the ghost
    layer supplies g_j(q + c_a) on links that leave the mesh through a wall or a
    far-field face, and the periodic wrap supplies it across periodic faces.
    """
    lat = mesh.lat
    d = mesh.d
    L = box_layers(mesh)
    g = bas["g"]
    g0 = _view(g, 2, [0] * d, L, 0)
    gco0 = _view(bas["gco"], 2, [0] * d, L, 0)
    out = np.zeros((lat.Q, d) + mesh.shape)
    for a in range(lat.Q):
        c = lat.c[a]
        gs = _view(g, 2, list(c), L, 0)
        e_here = np.einsum("j,jk...->k...", lat.cf[a], g0)
        e_there = np.einsum("j,jk...->k...", lat.cf[a], gs)
        out[a] = np.einsum("k...,ik...->i...", e_there - e_here, gco0)
    return out


def theta(mesh, bas, offset):
    """Theta^i_j(q + offset, q) = [g_j(q + offset) - g_j(q)] . g^i(q) on real
    cells (eq. (gamma)); shape (i, j, *n).  Used by the geometry pins."""
    d = mesh.d
    L = box_layers(mesh)
    g = bas["g"]
    g0 = _view(g, 2, [0] * d, L, 0)
    gs = _view(g, 2, list(offset), L, 0)
    gco0 = _view(bas["gco"], 2, [0] * d, L, 0)
    return np.einsum("jk...,ik...->ij...", gs - g0, gco0)


def real(field, lead, d, layers=1):
    """The real-cell part of a field given on the box q in [-layers, n + layers)."""
    return _view(field, lead, [0] * d, layers, 0)


class Geometry:
    """Everything the dynamics needs, on real cells (eq. (gamma) and before).

    g (d, d, *n), J (*n), gco (d, d, *n), gup (d, d, *n), A (Q, d, *n),
    aext (d, *n): contravariant components of a Euclidean body acceleration G,
    a_ext^i = G . g^i (the body force is a reading; the paper has none).
    """

    def __init__(self, mesh, body_force=None):
        self.mesh = mesh
        self.lat = mesh.lat
        d = mesh.d
        bas = basis(mesh)
        L = box_layers(mesh)
        self.box = bas
        self.g = real(bas["g"], 2, d, L)
        self.J = real(bas["J"], 0, d, L)
        self.gco = real(bas["gco"], 2, d, L)
        self.gup = real(bas["gup"], 2, d, L)
        self.A = link_coefficients(mesh, bas)
        G = np.zeros(d) if body_force is None else np.asarray(body_force, dtype=np.float64)[:d]
        self.G = G
        self.aext = np.einsum("k,ik...->i...", G, self.gco)

    def report(self):
        """Diagnostics: min/max J, range of g^{ij} eigenvalues, the smallest
        rest-equilibrium ratio f^eq(rho=1, U=0)/w, and max |A|."""
        lat = self.lat
        d = self.mesh.d
        gup = np.moveaxis(self.gup.reshape(d, d, -1), -1, 0)
        ev = np.linalg.eigvalsh(gup)
        H2 = np.einsum("ai,aj->aij", lat.cf, lat.cf) / lat.T0 - np.eye(d)[None]
        dev = self.gup - np.eye(d).reshape((d, d) + (1,) * d)
        ratio = 1.0 + 0.5 * np.einsum("aij,ij...->a...", H2, dev)
        return {
            "min_J": float(self.J.min()), "max_J": float(self.J.max()),
            "min_gup_eig": float(ev.min()), "max_gup_eig": float(ev.max()),
            "min_rest_feq_over_w": float(ratio.min()),
            "max_abs_A": float(np.abs(self.A).max()),
        }
