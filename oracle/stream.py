"""One-to-one advection (Sec. 2.2, eq. (adv)): N_a(q + c_a, t + 1) = N'_a(q, t),
written as a pull: N_a(q, t + 1) = N'_a(q - c_a, t).

Readings for links whose source q - c_a lies outside the index box (the paper
puts boundary treatment out of its scope):
* periodic axis: the index wraps;
* wall face: halfway bounce-back, N_a(q, t + 1) = N'_opp(a)(q, t);
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


def sources(mesh):
    """Per direction a: (flat source index (*n), kind (*n)) where kind is
    INTERIOR, WALL or FARFIELD; for WALL/FARFIELD links the index is the cell
    itself (the bounce-back slot)."""
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
        flat = np.where(kind == INTERIOR, flat, own)
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
