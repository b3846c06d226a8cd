"""Thin ctypes binding of libvlbm.so (include/vlbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory and the current HIP stream.  The library is
loaded from this package directory; if it is missing the import fails loudly
(there is no CPU fallback).

The module exposes the C functions under their C names (vlbm_mesh_create, ...),
raising VlbmError on a non-zero status, and two small handle classes, Mesh and
Sim, that own the C handles and the torch tensors passed across the boundary.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libvlbm.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is not built: run __graft_entry__.build() "
                      "or python -m paper_2401_17183_amd.build")
_lib = C.CDLL(LIBPATH)

D2Q9, D3Q19, D2Q21, D3Q39 = 0, 1, 2, 3
FP64, FP32, FP16S, BF16S, FP32C = 0, 1, 2, 3, 4
PERIODIC, WALL, FARFIELD = 0, 1, 2
OK, ERR_ARG, ERR_MESH, ERR_NOMEM, ERR_DEVICE, ERR_NOCONVERGE, ERR_STATE, ERR_NONFINITE, ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
BATCH_PERSISTENT_GRAPH, BATCH_PERSISTENT, BATCH_EAGER, BATCH_EAGER_GRAPH = 0, 1, 2, 3
LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19, "D2Q21": D2Q21, "D3Q39": D3Q39}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S, "bf16s": BF16S, "fp32c": FP32C}


class VlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class vlbm_topology(C.Structure):
    _fields_ = [("face", (C.c_int32 * 2) * 3), ("wrap", (C.c_double * 3) * 3)]


class vlbm_geom_report(C.Structure):
    _fields_ = [("min_J", C.c_double), ("max_J", C.c_double), ("min_gup_eig", C.c_double),
                ("max_gup_eig", C.c_double), ("min_rest_feq_over_w", C.c_double), ("max_abs_A", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vlbm_params(C.Structure):
    _fields_ = [("tau", C.c_double), ("body_force", C.c_double * 3), ("rho_inf", C.c_double),
                ("u_inf", C.c_double * 3), ("precision", C.c_int32), ("fp_max_iter", C.c_int32),
                ("fp_tol", C.c_double), ("audit_every", C.c_int32), ("stream_only", C.c_int32),
                ("tau_g", C.c_double), ("rebase_every", C.c_int32)]


class vlbm_audit(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("mom_I", C.c_double * 3),
                ("wall_impulse", C.c_double * 3), ("force_impulse", C.c_double * 3), ("residual", C.c_double),
                ("max_fp_iters", C.c_int32), ("nonfinite", C.c_int32), ("negative", C.c_int32),
                ("unconverged", C.c_int32)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = np.array(list(v)) if isinstance(v, C.Array) else v
        return out


class vlbm_conv_desc(C.Structure):
    _fields_ = [("batch", C.c_int), ("height", C.c_int), ("width", C.c_int), ("c_in", C.c_int),
                ("c_skip", C.c_int), ("upsample", C.c_int), ("stride", C.c_int), ("c_out", C.c_int),
                ("relu", C.c_int)]


class vlbm_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


_P = C.c_void_p
_SIGS = {
    "vlbm_last_error": (C.c_char_p, []),
    "vlbm_lattice_info": (C.c_int, [C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double)]),
    "vlbm_mesh_create": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(vlbm_topology), C.c_double, C.POINTER(_P)]),
    "vlbm_mesh_destroy": (C.c_int, [_P]),
    "vlbm_geometry_precompute": (C.c_int, [_P, _P, C.POINTER(vlbm_geom_report)]),
    "vlbm_geometry_precompute_noalloc": (C.c_int, [_P, _P, C.POINTER(vlbm_geom_report)]),
    "vlbm_geometry_fields": (C.c_int, [_P, _P, _P, _P, _P]),
    "vlbm_init": (C.c_int, [_P, C.POINTER(vlbm_params), _P, _P, _P, C.POINTER(_P)]),
    "vlbm_step": (C.c_int, [_P, C.c_int64]),
    "vlbm_sync": (C.c_int, [_P]),
    "vlbm_step_moving": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "vlbm_step_stats": (C.c_int, [_P, C.c_int, C.POINTER(C.c_uint64)]),
    "vlbm_kernel_timing": (C.c_int, [_P, C.c_int, C.POINTER(C.c_double)]),
    "vlbm_membench": (C.c_int, [C.c_int, C.c_int, C.c_size_t, C.c_int, _P, C.POINTER(C.c_double),
                                C.POINTER(C.c_int)]),
    "vlbm_set_fixed_point": (C.c_int, [_P, C.c_int32, C.c_double]),
    "vlbm_moments": (C.c_int, [_P, _P, _P, _P]),
    "vlbm_populations": (C.c_int, [_P, _P]),
    "vlbm_set_populations": (C.c_int, [_P, _P]),
    "vlbm_audit_now": (C.c_int, [_P]),
    "vlbm_audits": (C.c_int, [_P, C.POINTER(vlbm_audit), C.c_int, C.POINTER(C.c_int)]),
    "vlbm_save": (C.c_int, [_P, _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "vlbm_restore": (C.c_int, [_P, _P, C.c_size_t]),
    "vlbm_sim_step_count": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "vlbm_sim_destroy": (C.c_int, [_P]),
    "vlbm_reinit": (C.c_int, [_P, _P, _P]),
    "vlbm_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(vlbm_params), C.c_int, _P, C.POINTER(_P)]),
    "vlbm_batch_member": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "vlbm_batch_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(_P),
                                  C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "vlbm_batch_set_mode": (C.c_int, [_P, C.c_int]),
    "vlbm_batch_config": (C.c_int, [_P, C.c_int, C.c_int]),
    "vlbm_batch_step": (C.c_int, [_P, C.c_int64]),
    "vlbm_batch_sync": (C.c_int, [_P]),
    "vlbm_batch_autotune": (C.c_int, [_P, C.c_int, C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "vlbm_batch_destroy": (C.c_int, [_P]),
    "vlbm_batch_residuals": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "vlbm_batch_set_active": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "vlbm_conv2d_forward": (C.c_int, [C.POINTER(vlbm_conv_desc), _P, _P, _P, _P, _P, _P, _P]),
    "vlbm_conv2d_backward_data": (C.c_int, [C.POINTER(vlbm_conv_desc), _P, _P, _P, _P, _P]),
    "vlbm_conv2d_backward_weight": (C.c_int, [C.POINTER(vlbm_conv_desc), _P, _P, _P, _P, _P, _P]),
    "vlbm_conv2d_pack_weights": (C.c_int, [C.POINTER(vlbm_conv_desc), _P, _P, _P, _P]),
    "vlbm_adam_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(vlbm_adam), C.c_int64, _P]),
    "vlbm_surrogate_param_count": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int64)]),
    "vlbm_surrogate_create": (C.c_int, [C.c_int, C.c_int, C.c_int, _P, _P, C.POINTER(_P)]),
    "vlbm_surrogate_forward": (C.c_int, [_P, _P, C.c_int, _P]),
    "vlbm_surrogate_gradient": (C.c_int, [_P, _P, _P, C.c_int, C.POINTER(C.c_double), _P]),
    "vlbm_surrogate_adam": (C.c_int, [_P, C.POINTER(vlbm_adam)]),
    "vlbm_surrogate_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.POINTER(vlbm_adam), C.POINTER(C.c_double)]),
    "vlbm_surrogate_params": (C.c_int, [_P, _P, C.POINTER(C.c_int64)]),
    "vlbm_surrogate_destroy": (C.c_int, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def vlbm_last_error():
    return _lib.vlbm_last_error().decode()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise VlbmError(rc, vlbm_last_error())
    return rc


def _wrap(name):
    f = getattr(_lib, name)

    def call(*args, allow=()):
        return _check(f(*args), allow)
    call.__name__ = name
    call.__doc__ = f"ctypes call of {name} (include/vlbm.h); raises VlbmError on failure"
    return call


for _name in _SIGS:
    if _name != "vlbm_last_error":
        globals()[_name] = _wrap(_name)


def lattice_info(lattice):
    Q, d = C.c_int32(), C.c_int32()
    vlbm_lattice_info(lattice, C.byref(Q), C.byref(d), None, None)
    c = (C.c_int32 * (Q.value * d.value))()
    w = (C.c_double * Q.value)()
    vlbm_lattice_info(lattice, C.byref(Q), C.byref(d), c, w)
    return np.array(c[:]).reshape(Q.value, d.value), np.array(w[:])


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the library has no CPU path")
    return torch


def _stream_ptr(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(torch, a, shape=None):
    """Contiguous float64 device tensor from a numpy array / tensor."""
    t = torch.as_tensor(a, dtype=torch.float64)
    if shape is not None:
        t = t.reshape(shape)
    return t.to("cuda").contiguous()


def _is_tensor(a):
    return type(a).__module__.startswith("torch")


def _ready(torch):
    """Finish torch's pending work on its current stream: buffers allocated or
    filled there are then safe to hand to a library call on another stream
    (batch members run on the batch's own stream)."""
    torch.cuda.current_stream().synchronize()


class Mesh:
    """A mesh handle: coordinates in, FP64 geometry precomputed on the device."""

    def __init__(self, lattice, n, coords, faces, wrap, dx, precompute=True):
        self.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
        self.d = 2 if self.lattice in (D2Q9, D2Q21) else 3
        self.Q = {D2Q9: 9, D3Q19: 19, D2Q21: 21, D3Q39: 39}[self.lattice]
        n = tuple(int(v) for v in n)
        self.n = n
        self.ncells = int(np.prod(n))
        nn = (C.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
        topo = vlbm_topology()
        for i in range(self.d):
            for f in range(2):
                topo.face[i][f] = int(faces[i][f])
            for k in range(self.d):
                topo.wrap[i][k] = float(wrap[i][k])
        h = _P()
        torch = _torch() if _is_tensor(coords) else None
        if torch is not None and coords.is_cuda:   # device coordinates stay on the device
            X = coords.detach().to(torch.float64).contiguous()
            _ready(torch)
            ptr = C.cast(C.c_void_p(X.data_ptr()), C.POINTER(C.c_double))
        else:
            X = np.ascontiguousarray(coords.cpu().numpy() if torch is not None else coords, dtype=np.float64)
            ptr = X.ctypes.data_as(C.POINTER(C.c_double))
        vlbm_mesh_create(self.lattice, nn, ptr, C.byref(topo), float(dx), C.byref(h))
        self.h = h
        self.report = None
        if precompute:
            self.precompute()

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w["lattice"], w["n"], w["coords"], w["faces"], w["wrap"], w["dx"], **kw)

    def precompute(self, noalloc=False):
        torch = _torch()
        rep = vlbm_geom_report()
        fn = vlbm_geometry_precompute_noalloc if noalloc else vlbm_geometry_precompute
        fn(self.h, _stream_ptr(torch), C.byref(rep))
        self.report = rep.as_dict()
        return self.report

    def fields(self):
        """FP64 geometry as torch tensors: J, gup (d,d), A (Q,d), g (d,d) per cell."""
        torch = _torch()
        nc, d, Q = self.ncells, self.d, self.Q
        J = torch.empty(nc, dtype=torch.float64, device="cuda")
        gup = torch.empty(d * d * nc, dtype=torch.float64, device="cuda")
        A = torch.empty(Q * d * nc, dtype=torch.float64, device="cuda")
        g = torch.empty(d * d * nc, dtype=torch.float64, device="cuda")
        vlbm_geometry_fields(self.h, _P(J.data_ptr()), _P(gup.data_ptr()), _P(A.data_ptr()), _P(g.data_ptr()))
        return {"J": J, "gup": gup.reshape(d, d, nc), "A": A.reshape(Q, d, nc), "g": g.reshape(d, d, nc)}

    def close(self):
        if getattr(self, "h", None):
            vlbm_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(tau, body_force=(0, 0, 0), rho_inf=1.0, u_inf=(0, 0, 0), precision=FP64, fp_max_iter=0,
                fp_tol=-1.0, audit_every=0, stream_only=False, tau_g=None, rebase_every=0):
    """Simulation parameters; tau_g None (or tau) is BGK, otherwise the general
    collision matrix whose non-hydrodynamic part relaxes at 1/tau_g."""
    p = vlbm_params()
    p.tau = float(tau)
    p.tau_g = 0.0 if tau_g is None else float(tau_g)
    p.rebase_every = int(rebase_every)
    bf = list(body_force) + [0.0] * (3 - len(body_force))
    ui = list(u_inf) + [0.0] * (3 - len(u_inf))
    for k in range(3):
        p.body_force[k] = float(bf[k])
        p.u_inf[k] = float(ui[k])
    p.rho_inf = float(rho_inf)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.fp_max_iter = int(fp_max_iter)
    p.fp_tol = float(fp_tol)
    p.audit_every = int(audit_every)
    p.stream_only = int(bool(stream_only))
    return p


class Sim:
    """A simulation handle on a Mesh (populations, packed geometry, audits)."""

    def __init__(self, mesh, params, rho=None, u=None):
        torch = _torch()
        self.mesh = mesh
        self.params = params
        nc, d = mesh.ncells, mesh.d
        r = _dev(torch, rho, (nc,)) if rho is not None else None
        v = _dev(torch, u, (d, nc)) if u is not None else None
        h = _P()
        vlbm_init(mesh.h, C.byref(params), _P(r.data_ptr()) if r is not None else None,
                  _P(v.data_ptr()) if v is not None else None, _stream_ptr(torch), C.byref(h))
        self.h = h
        self._stream = torch.cuda.current_stream().cuda_stream   # the stream the sim launches on

    def step(self, n=1):
        vlbm_step(self.h, int(n))

    def step_moving(self, coords_next, wrap_next=None):
        """One step with the mesh moving to coords_next (mesh layout; host
        array or device tensor) and periodic translations wrap_next (d x d)."""
        torch = _torch()
        X = _dev(torch, coords_next, (int(np.prod(np.shape(coords_next))),))
        wr = None
        if wrap_next is not None:
            w = np.zeros((3, 3))
            a = np.asarray(wrap_next, dtype=np.float64)
            w[: a.shape[0], : a.shape[1]] = a
            wr = (C.c_double * 9)(*w.ravel())
        if torch.cuda.current_stream().cuda_stream != self._stream:
            _ready(torch)   # coords_next may still be in flight on another stream
        vlbm_step_moving(self.h, _P(X.data_ptr()), wr)
        self._keep = X   # the call is asynchronous: keep the input alive until the next call

    def sync(self):
        """Wait for the enqueued steps; raises VlbmError(ERR_NOCONVERGE) when a
        step since the last report hit the fixed point's cap."""
        vlbm_sync(self.h)

    def kernel_timing(self, enable=False):
        """Kernel durations recorded since the last read (then cleared), and
        turn the recording on or off for the following steps:
        {step_ms, step_launches, rebase_ms, rebase_launches, basis_ms,
        basis_launches} (the last two: the geometry kernel of moving steps)."""
        out = (C.c_double * 6)()
        vlbm_kernel_timing(self.h, int(bool(enable)), out)
        return {"step_ms": out[0], "step_launches": int(out[1]), "rebase_ms": out[2],
                "rebase_launches": int(out[3]), "basis_ms": out[4], "basis_launches": int(out[5])}

    def set_fixed_point(self, max_iter=0, tol=-1.0):
        vlbm_set_fixed_point(self.h, int(max_iter), float(tol))

    def step_stats(self, enable=False):
        """Fixed-point statistics since the last read (then reset), and turn
        their collection on or off for the following steps:
        {iters_per_cell, wave_max_iters, cell_steps, wave_steps}."""
        out = (C.c_uint64 * 4)()
        vlbm_step_stats(self.h, int(bool(enable)), out)
        cells, waves = int(out[2]), int(out[3])
        return {"iters_per_cell": out[0] / cells if cells else float("nan"),
                "wave_max_iters": out[1] / waves if waves else float("nan"),
                "cell_steps": cells, "wave_steps": waves}

    @property
    def t(self):
        v = C.c_int64()
        vlbm_sim_step_count(self.h, C.byref(v))
        return v.value

    def moments(self, with_U=False):
        torch = _torch()
        nc, d = self.mesh.ncells, self.mesh.d
        rho = torch.empty(nc, dtype=torch.float64, device="cuda")
        u = torch.empty(d * nc, dtype=torch.float64, device="cuda")
        U = torch.empty(d * nc, dtype=torch.float64, device="cuda") if with_U else None
        _ready(torch)
        vlbm_moments(self.h, _P(rho.data_ptr()), _P(u.data_ptr()), _P(U.data_ptr()) if U is not None else None)
        out = {"rho": rho, "u": u.reshape(d, nc)}
        if U is not None:
            out["U"] = U.reshape(d, nc)
        return out

    def populations(self):
        torch = _torch()
        Q, nc = self.mesh.Q, self.mesh.ncells
        N = torch.empty(Q * nc, dtype=torch.float64, device="cuda")
        _ready(torch)
        vlbm_populations(self.h, _P(N.data_ptr()))
        return N.reshape(Q, nc)

    def set_populations(self, N):
        torch = _torch()
        t = _dev(torch, N, (self.mesh.Q * self.mesh.ncells,))
        _ready(torch)
        vlbm_set_populations(self.h, _P(t.data_ptr()))

    def audit_now(self):
        vlbm_audit_now(self.h)

    def reinit(self, rho=None, u=None):
        torch = _torch()
        nc, d = self.mesh.ncells, self.mesh.d
        r = _dev(torch, rho, (nc,)) if rho is not None else None
        v = _dev(torch, u, (d, nc)) if u is not None else None
        _ready(torch)
        vlbm_reinit(self.h, _P(r.data_ptr()) if r is not None else None, _P(v.data_ptr()) if v is not None else None)

    def audits(self, cap=4096, allow_nonfinite=True):
        buf = (vlbm_audit * cap)()
        n = C.c_int()
        vlbm_audits(self.h, buf, cap, C.byref(n), allow=(ERR_NONFINITE,) if allow_nonfinite else ())
        return [buf[i].as_dict() for i in range(n.value)]

    def save(self):
        used = C.c_size_t()
        vlbm_save(self.h, None, 0, C.byref(used))
        buf = C.create_string_buffer(used.value)
        vlbm_save(self.h, buf, used.value, C.byref(used))
        return bytes(buf.raw[: used.value])

    def restore(self, blob):
        b = C.create_string_buffer(blob, len(blob))
        vlbm_restore(self.h, b, len(blob))

    def close(self):
        if getattr(self, "h", None):
            vlbm_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(Sim):
    """A borrowed member of a Batch (the batch owns and frees it)."""

    def __init__(self, mesh, params, h):
        self.mesh = mesh
        self.params = params
        self.h = h
        self._stream = None   # members run on the batch's own stream

    def close(self):
        self.h = None


class Batch:
    """Many meshes advanced together (one persistent launch per step)."""

    def __init__(self, meshes, params, stream=None):
        _torch()
        n = len(meshes)
        hs = (_P * n)(*[m.h for m in meshes])
        ps = (vlbm_params * n)(*params)
        h = _P()
        vlbm_batch_create(hs, ps, n, _P(stream) if stream else None, C.byref(h))
        self.h = h
        self.meshes = list(meshes)
        self.params = list(params)
        self.members = []
        for i in range(n):
            mh = _P()
            vlbm_batch_member(self.h, i, C.byref(mh))
            self.members.append(_Member(meshes[i], params[i], mh))

    def info(self):
        cnt, cells, st, bl, gp = C.c_int(), C.c_int64(), _P(), C.c_int(), C.c_int()
        vlbm_batch_info(self.h, C.byref(cnt), C.byref(cells), C.byref(st), C.byref(bl), C.byref(gp))
        return {"count": cnt.value, "cells": cells.value, "stream": st.value, "block": bl.value,
                "grid_per_cu": gp.value}

    def set_mode(self, mode):
        vlbm_batch_set_mode(self.h, int(mode))

    def config(self, block, grid_per_cu):
        vlbm_batch_config(self.h, int(block), int(grid_per_cu))

    def step(self, n=1):
        vlbm_batch_step(self.h, int(n))

    def sync(self):
        vlbm_batch_sync(self.h)

    def residuals(self):
        """Audit every member now; numpy array of steady-state residuals
        ||u - u_prev|| / ||u|| against each member's previous audit (NaN at the first)."""
        out = (C.c_double * len(self.members))()
        vlbm_batch_residuals(self.h, out)
        return np.array(out[:])

    def set_active(self, active=None):
        """Members stepped by step(): a boolean sequence of length count (None = all)."""
        if active is None:
            vlbm_batch_set_active(self.h, None)
            return
        a = (C.c_int32 * len(self.members))(*[1 if x else 0 for x in active])
        vlbm_batch_set_active(self.h, a)

    def autotune(self, trial_steps=20, cache_path=None):
        bl, gp = C.c_int(), C.c_int()
        vlbm_batch_autotune(self.h, int(trial_steps), cache_path.encode() if cache_path else None,
                            C.byref(bl), C.byref(gp))
        return bl.value, gp.value

    def close(self):
        if getattr(self, "h", None):
            for m in self.members:
                m.h = None
            vlbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def membench(kind, nontemporal=False, bytes_=2 << 30, reps=10):
    """Best STREAM-style bandwidth in GB/s (kind "read", "write" or "copy")
    and the grid of that launch, on torch's current stream."""
    torch = _torch()
    k = {"read": 0, "write": 1, "copy": 2}[kind]
    g = C.c_double()
    grid = C.c_int()
    vlbm_membench(k, int(bool(nontemporal)), int(bytes_), int(reps), _stream_ptr(torch), C.byref(g), C.byref(grid))
    return g.value, grid.value


def _ptr(t):
    return None if t is None else _P(t.data_ptr())


def conv_desc(batch, height, width, c_in, c_out, c_skip=0, upsample=False, stride=1, relu=True):
    return vlbm_conv_desc(batch, height, width, c_in, c_skip, int(bool(upsample)), stride, c_out, int(bool(relu)))


def _cur_stream():
    return _stream_ptr(_torch())


def conv2d_forward(d, x, skip, w, bias, y_bf16=None, y_f32=None):
    """BF16 tensors as torch.bfloat16 (raw words), FP32 as torch.float32; async
    on torch's current stream."""
    vlbm_conv2d_forward(C.byref(d), _ptr(x), _ptr(skip), _ptr(w), _ptr(bias), _ptr(y_bf16), _ptr(y_f32),
                        _cur_stream())


def conv2d_backward_data(d, gy, wt, gx=None, gskip=None):
    vlbm_conv2d_backward_data(C.byref(d), _ptr(gy), _ptr(wt), _ptr(gx), _ptr(gskip), _cur_stream())


def conv2d_backward_weight(d, x, skip, gy, gw, gb):
    vlbm_conv2d_backward_weight(C.byref(d), _ptr(x), _ptr(skip), _ptr(gy), _ptr(gw), _ptr(gb), _cur_stream())


def conv2d_pack_weights(d, w, w_bf16, wt_bf16):
    vlbm_conv2d_pack_weights(C.byref(d), _ptr(w), _ptr(w_bf16), _ptr(wt_bf16), _cur_stream())


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    hp = vlbm_adam(lr, beta1, beta2, eps)
    vlbm_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), C.byref(hp), int(step), _cur_stream())


def surrogate_param_count(height, width):
    n = C.c_int64()
    vlbm_surrogate_param_count(int(height), int(width), C.byref(n))
    return n.value


class Surrogate:
    """The BF16-MFMA encoder-decoder (include/vlbm.h).  Inputs and outputs are
    torch float32 device tensors [batch][height][width][3]; runs on torch's
    current stream at creation."""

    def __init__(self, height, width, max_batch, params):
        torch = _torch()
        self.height, self.width, self.max_batch = int(height), int(width), int(max_batch)
        self.nparams = surrogate_param_count(height, width)
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1).to("cuda").contiguous()
        if p.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {p.numel()}")
        h = _P()
        _ready(torch)
        vlbm_surrogate_create(self.height, self.width, self.max_batch, _ptr(p), _stream_ptr(torch), C.byref(h))
        self.h = h
        torch.cuda.current_stream().synchronize()

    def _in(self, x, channels=3):
        torch = _torch()
        t = torch.as_tensor(x, dtype=torch.float32).to("cuda").contiguous()
        if t.dim() != 4 or tuple(t.shape[1:]) != (self.height, self.width, channels):
            raise ValueError(f"expected [batch][{self.height}][{self.width}][{channels}], got {tuple(t.shape)}")
        return t

    def forward(self, x):
        torch = _torch()
        x = self._in(x)
        y = torch.empty_like(x)
        _ready(torch)
        vlbm_surrogate_forward(self.h, _ptr(x), x.shape[0], _ptr(y))
        return y

    def gradient(self, x, target, with_grad=True):
        torch = _torch()
        x, t = self._in(x), self._in(target)
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda") if with_grad else None
        loss = C.c_double()
        _ready(torch)
        vlbm_surrogate_gradient(self.h, _ptr(x), _ptr(t), x.shape[0], C.byref(loss), _ptr(g))
        return loss.value, g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        hp = vlbm_adam(lr, beta1, beta2, eps)
        vlbm_surrogate_adam(self.h, C.byref(hp))

    def train_step(self, x, target, lr, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=True):
        torch = _torch()
        x, t = self._in(x), self._in(target)
        hp = vlbm_adam(lr, beta1, beta2, eps)
        loss = C.c_double()
        _ready(torch)
        vlbm_surrogate_train_step(self.h, _ptr(x), _ptr(t), x.shape[0], C.byref(hp),
                                  C.byref(loss) if want_loss else None)
        return loss.value if want_loss else None

    def params(self):
        torch = _torch()
        out = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        step = C.c_int64()
        _ready(torch)
        vlbm_surrogate_params(self.h, _ptr(out), C.byref(step))
        return out, step.value

    def close(self):
        if getattr(self, "h", None):
            vlbm_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
