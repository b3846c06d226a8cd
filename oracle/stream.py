"""One-to-one advection (Sec. 2.2, eq. (adv)): N_a(q + c_a, t + 1) = N'_a(q, t),
written as a pull: N_a(q, t + 1) = N'_a(q - c_a, t).

Readings for links whose source q - c_a lies outside the index box (the paper
puts boundary treatment out of its scope):
* periodic axis: the index wraps;
* wall face: halfway bounce-back, N_a(q, t + 1) = N'_opp(a)(q, t);
* wall face, links longer than one cell (D2Q21, D3Q39; walls on one axis
  i only): the particle that arrives at q along c_a left a cell q_s along
  -c_a, met the wall (half a cell beyond the last real cell), reversed and
  finished the time step: N_a(q, t + 1) = N'_opp(a)(q_s, t).  With d the
  distance of q_s from the wall in cells, its path gives
  q_s^i = |c^i| - 1 - q^i at the low face (2 n_i - 1 - |c^i| - q^i at the
  high face) and q_s^j = q^j - c^j (1 - (2 d + 1) / |c^i|) on the other axes
  (integer on these lattices, whose diagonal links have |c^j| = |c^i|).  For a
  one-cell link q_s = q, the rule above;
* far-field face: N_a(q, t + 1) = N_inf_a(q), an imposed population;
* a link leaving through both a far-field and a wall face counts as far-field.

Pinned by: streaming alone is a permutation (every post-collision population
lands in exactly one slot), n pure-streaming steps on an n-periodic axis
return the state unchanged, bit for bit, and a uniform state equal to the
far-field state stays unchanged on a uniform lattice with far-field faces
(tests/test_oracle_stream.py).
"""
import numpy as np

from .geometry import PERIODIC, WALL, FARFIELD

INTERIOR = 0


def wall_source(mesh, a, q, i, mask):
    """The cell q_s whose opposite population reaches q along direction a
    after reflection at the wall of axis i (the multi-cell rule above);
    q (list of index arrays), returns the list of q_s index arrays (valid
    where mask, the links that do meet the wall, is set)."""
    c = mesh.lat.c[a]
    ci = int(c[i])
    k = abs(ci)
    n = mesh.n[i]
    qs_i = (k - 1 - q[i]) if ci > 0 else (2 * n - 1 - k - q[i])
    dist = qs_i if ci > 0 else n - 1 - qs_i
    out = []
    for j in range(mesh.d):
        if j == i:
            out.append(qs_i)
            continue
        cj = int(c[j])
        num = cj * (k - 2 * dist - 1)            # c^j (1 - (2 d + 1) / |c^i|) |c^i|
        assert np.all((num % k)[mask] == 0)
        sj = q[j] - num // k
        out.append(np.mod(sj, mesh.n[j]) if mesh.periodic(j) else sj)
    return out


def sources(mesh):
    """Per direction a: (flat source index (*n), kind (*n)) where kind is
    INTERIOR, WALL or FARFIELD; for FARFIELD links the index is the cell
    itself, for WALL links the cell whose opposite population bounces into q
    (the cell itself for one-cell links)."""
    lat = mesh.lat
    d = mesh.d
    out = []
    grids = np.meshgrid(*[np.arange(mesh.n[i]) for i in reversed(range(d))], indexing="ij")
    q = [grids[d - 1 - i] for i in range(d)]  # q[i] has the real-cell shape
    for a in range(lat.Q):
        s = []
        kind = np.zeros(mesh.shape, dtype=np.int64)
        for i in range(d):
            si = q[i] - lat.c[a][i]
            if mesh.periodic(i):
                si = np.mod(si, mesh.n[i])
            else:
                lo, hi = mesh.faces[i]
                below = si < 0
                above = si >= mesh.n[i]
                for m, f in ((below, lo), (above, hi)):
                    if f == FARFIELD:
                        kind[m] = FARFIELD
                    elif f == WALL:
                        kind[m & (kind != FARFIELD)] = WALL
                si = np.clip(si, 0, mesh.n[i] - 1)
            s.append(si)
        flat = np.zeros(mesh.shape, dtype=np.int64)
        for i in reversed(range(d)):
            flat = flat * mesh.n[i] + s[i]
        own = np.arange(mesh.ncells).reshape(mesh.shape)
        bounce = own
        if lat.speed > 1 and np.any(kind == WALL):
            wi = [i for i in range(d) if not mesh.periodic(i)][0]
            qs = wall_source(mesh, a, q, wi, kind == WALL)
            bounce = np.zeros(mesh.shape, dtype=np.int64)
            for i in reversed(range(d)):
                bounce = bounce * mesh.n[i] + np.where(kind == WALL, qs[i], 0)
        flat = np.where(kind == INTERIOR, flat, np.where(kind == WALL, bounce, own))
        out.append((flat, kind))
    return out


def stream(mesh, Np, N_inf=None, src=None):
    """Pull-stream post-collision populations Np (Q, *n) -> arrived N (Q, *n)."""
    lat = mesh.lat
    if src is None:
        src = sources(mesh)
    flatNp = Np.reshape(lat.Q, -1)
    N = np.empty_like(Np)
    for a in range(lat.Q):
        idx, kind = src[a]
        v = flatNp[a][idx]
        v = np.where(kind == WALL, flatNp[lat.opp[a]][idx], v)
        if N_inf is not None:
            v = np.where(kind == FARFIELD, N_inf[a], v)
        N[a] = v
    return N
