"""ctypes binding of liblasto.so (the C ABI in include/lasto.h).

Argument marshalling only: every step of the Hartree path runs in the HIP
kernels behind the C ABI. torch supplies device memory and the stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblasto.so")

OK, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_NOT_CONVERGED, ERR_DIVERGED, ERR_STATE = range(7)
# points one call of lasto_sphere_interp_noalloc may take (LASTO_NOALLOC_MAX_POINTS)
NOALLOC_MAX_POINTS = 32768


class LastoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("lasto status %d: %s" % (status, msg))
        self.status = status


class Atom(C.Structure):
    _fields_ = [
        ("center", C.c_double * 3),
        ("radius", C.c_double),
        ("q", C.c_double),
        ("kind", C.c_int),
        ("lmax", C.c_int),
        ("width", C.c_double),
        ("rho_R", C.c_double),
        ("drho_R", C.c_double),
        ("alpha", C.c_double),
        ("clm", C.c_double * 24),
    ]


class Shell(C.Structure):
    _fields_ = [("n", C.c_int), ("l", C.c_int), ("zeta", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double),
        ("max_iters", C.c_int),
        ("nu1", C.c_int),
        ("nu2", C.c_int),
        ("method", C.c_int),
        ("precision", C.c_int),
        ("inner_iters", C.c_int),
        ("guess", C.c_int),
        ("bc", C.c_int),
        ("lmax_bc", C.c_int),
        ("debug_nan_iter", C.c_int),
        ("profile", C.c_int),
        ("inner_first", C.c_int),
        ("coarse", C.c_int),
        ("fallback", C.c_int),
        ("n_atoms", C.c_int),
        ("atoms", C.c_void_p),
        ("guess_net", C.c_void_p),
        ("coarse_net", C.c_void_p),
        ("coarse_net_level", C.c_int),
        ("inner_rate", C.c_double),
        ("graphs", C.c_int),
        ("nu_coarse", C.c_int),
        ("fused_sweeps", C.c_int),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int),
        ("vcycles", C.c_int),
        ("refinements", C.c_int),
        ("rel_resid", C.c_double),
        ("resid_hist", C.c_double * 128),
        ("moments", C.c_double * 25),
        ("ms_total", C.c_double),
        ("smooth_launches", C.c_int),
        ("smooth_ms", C.c_double),
        ("smooth_bytes", C.c_double),
        ("smooth_fp32", C.c_int),
        ("n_batch", C.c_int),
        ("batch_rel_resid", C.c_double * 16),
        ("coarse_level", C.c_int),
        ("fallback_used", C.c_int),
        ("guess_accepted", C.c_int),
        ("coarse_applied", C.c_int),
        ("coarse_accepted", C.c_int),
        ("ms_bc", C.c_double),
        ("ms_guess", C.c_double),
        ("ms_cycles", C.c_double),
        ("alg_bytes", C.c_double),
        ("inner_rate", C.c_double),
        ("rel_start", C.c_double),
    ]

    def as_dict(self) -> dict:
        n = min(self.iters, 128)
        return dict(iters=self.iters, vcycles=self.vcycles, refinements=self.refinements,
                    rel_resid=self.rel_resid, resid_hist=list(self.resid_hist[:n]),
                    moments=list(self.moments), ms_total=self.ms_total,
                    smooth_launches=self.smooth_launches, smooth_ms=self.smooth_ms,
                    smooth_bytes=self.smooth_bytes, smooth_fp32=self.smooth_fp32,
                    batch_rel_resid=list(self.batch_rel_resid[:max(self.n_batch, 1)]),
                    coarse_level=self.coarse_level, fallback_used=self.fallback_used,
                    guess_accepted=self.guess_accepted, coarse_applied=self.coarse_applied,
                    coarse_accepted=self.coarse_accepted, ms_bc=self.ms_bc, ms_guess=self.ms_guess,
                    ms_cycles=self.ms_cycles, alg_bytes=self.alg_bytes, inner_rate=self.inner_rate,
                    rel_start=self.rel_start)


# exported names, in header order
SYMBOLS = [
    "lasto_status_string", "lasto_last_error", "lasto_mesh_graded_1d", "lasto_grid_create",
    "lasto_grid_destroy", "lasto_grid_levels", "lasto_grid_level_shape", "lasto_grid_level_nodes",
    "lasto_pseudo_density",
    "lasto_solve_opts_default", "lasto_poisson_solve", "lasto_sphere_interp", "lasto_sphere_interp_noalloc",
    "lasto_spheres_create", "lasto_spheres_destroy", "lasto_sphere_density_terms", "lasto_sphere_project", "lasto_sphere_radial",
    "lasto_sphere_energy", "lasto_interstitial_density", "lasto_matrix_elements", "lasto_fdm_solve",
    "lasto_fdm_axis", "lasto_apply", "lasto_rb_sweep", "lasto_smooth", "lasto_stream_probe", "lasto_boundary_values", "lasto_analytic_guess",
    "lasto_net_create", "lasto_net_destroy", "lasto_net_set_grid",
    "lasto_net_param_count", "lasto_net_get_params", "lasto_net_set_params", "lasto_net_get_grads",
    "lasto_net_save", "lasto_net_load", "lasto_net_get_config", "lasto_net_tensor",
    "lasto_net_features", "lasto_net_forward", "lasto_net_backward", "lasto_net_adam_step",
    "lasto_net_train_step", "lasto_learned_guess", "lasto_learned_correction", "lasto_coarse_pair", "lasto_net_correction_features",
]


class NetConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int),
        ("ny", C.c_int),
        ("nz", C.c_int),
        ("ch", C.c_int * 4),
        ("seed", C.c_ulonglong),
        ("rho_scale", C.c_double),
        ("pot_scale", C.c_double),
        ("h_ref", C.c_double),
        ("out_scale", C.c_double),
    ]

_lib = None


def load():
    """Load liblasto.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblasto.so is not built; run __graft_entry__.build() "
                           "(python paper_0806_1723_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    P, i, d = C.c_void_p, C.c_int, C.c_double
    L.lasto_status_string.argtypes = [i]
    L.lasto_status_string.restype = C.c_char_p
    L.lasto_last_error.argtypes = []
    L.lasto_last_error.restype = C.c_char_p
    L.lasto_mesh_graded_1d.argtypes = [d, d, i, P, i, d, d, d, d, P, P, P]
    L.lasto_mesh_graded_1d.restype = i
    L.lasto_grid_create.argtypes = [P, i, P, i, P, i, i, P, C.POINTER(P)]
    L.lasto_grid_create.restype = i
    L.lasto_grid_destroy.argtypes = [P]
    L.lasto_grid_destroy.restype = i
    L.lasto_grid_levels.argtypes = [P, C.POINTER(i)]
    L.lasto_grid_levels.restype = i
    L.lasto_grid_level_shape.argtypes = [P, i, P]
    L.lasto_grid_level_shape.restype = i
    L.lasto_grid_level_nodes.argtypes = [P, i, P, P, P]
    L.lasto_grid_level_nodes.restype = i
    L.lasto_pseudo_density.argtypes = [P, i, P, P, i, P, P]
    L.lasto_pseudo_density.restype = i
    L.lasto_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
    L.lasto_solve_opts_default.restype = None
    L.lasto_poisson_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]
    L.lasto_poisson_solve.restype = i
    L.lasto_sphere_interp.argtypes = [P, P, i, P, P, i, P, P]
    L.lasto_sphere_interp.restype = i
    L.lasto_sphere_interp_noalloc.argtypes = [P, P, i, P, P, i, P, P]
    L.lasto_sphere_interp_noalloc.restype = i
    L.lasto_spheres_create.argtypes = [P, i, P, P, P, i, i, i, d, C.POINTER(P)]
    L.lasto_spheres_create.restype = i
    L.lasto_spheres_destroy.argtypes = [P]
    L.lasto_spheres_destroy.restype = i
    L.lasto_sphere_density_terms.argtypes = [P, P, i, P]
    L.lasto_sphere_density_terms.restype = i
    L.lasto_sphere_project.argtypes = [P, P, P]
    L.lasto_sphere_project.restype = i
    L.lasto_sphere_radial.argtypes = [P, P, P, P]
    L.lasto_sphere_radial.restype = i
    L.lasto_sphere_energy.argtypes = [P, P, P, P, P, P]
    L.lasto_sphere_energy.restype = i
    L.lasto_interstitial_density.argtypes = [P, i, P, P, i, P, i, P, P, P]
    L.lasto_interstitial_density.restype = i
    L.lasto_matrix_elements.argtypes = [P, P, i, P, P, i, P, P, P]
    L.lasto_matrix_elements.restype = i
    L.lasto_fdm_solve.argtypes = [P, P, P, i, i, C.POINTER(SolveInfo)]
    L.lasto_fdm_solve.restype = i
    L.lasto_fdm_axis.argtypes = [P, i, P, P, P]
    L.lasto_fdm_axis.restype = i
    L.lasto_apply.argtypes = [P, P, P]
    L.lasto_apply.restype = i
    L.lasto_stream_probe.argtypes = [P, P, P, C.c_size_t, P]
    L.lasto_stream_probe.restype = i
    L.lasto_rb_sweep.argtypes = [P, P, P, P, i]
    L.lasto_rb_sweep.restype = i
    L.lasto_smooth.argtypes = [P, i, i, P, P, i, i, i, i, P]
    L.lasto_smooth.restype = i
    L.lasto_boundary_values.argtypes = [P, P, i, i, P, P]
    L.lasto_boundary_values.restype = i
    L.lasto_analytic_guess.argtypes = [P, i, P, P]
    L.lasto_analytic_guess.restype = i
    L.lasto_net_create.argtypes = [C.POINTER(NetConfig), P, C.POINTER(P)]
    L.lasto_net_create.restype = i
    L.lasto_net_destroy.argtypes = [P]
    L.lasto_net_destroy.restype = i
    L.lasto_net_param_count.argtypes = [P, C.POINTER(C.c_longlong)]
    L.lasto_net_param_count.restype = i
    for name in ("lasto_net_get_params", "lasto_net_set_params", "lasto_net_get_grads"):
        getattr(L, name).argtypes = [P, P, C.c_longlong]
        getattr(L, name).restype = i
    for name in ("lasto_net_save", "lasto_net_load"):
        getattr(L, name).argtypes = [P, C.c_char_p]
        getattr(L, name).restype = i
    L.lasto_net_get_config.argtypes = [P, C.POINTER(NetConfig), C.POINTER(C.c_longlong)]
    L.lasto_net_get_config.restype = i
    L.lasto_net_tensor.argtypes = [P, i, P, C.c_longlong, P]
    L.lasto_net_tensor.restype = i
    L.lasto_net_set_grid.argtypes = [P, i, i, i]
    L.lasto_net_set_grid.restype = i
    L.lasto_coarse_pair.argtypes = [P, P, P, P, i, i, P, P, C.POINTER(d), P]
    L.lasto_coarse_pair.restype = i
    L.lasto_net_features.argtypes = [P, P, P, P, P]
    L.lasto_net_features.restype = i
    L.lasto_net_forward.argtypes = [P, P, P]
    L.lasto_net_forward.restype = i
    L.lasto_net_backward.argtypes = [P, P, P, P, C.POINTER(d)]
    L.lasto_net_backward.restype = i
    L.lasto_net_adam_step.argtypes = [P, C.c_float]
    L.lasto_net_adam_step.restype = i
    L.lasto_net_train_step.argtypes = [P, P, P, P, C.c_float, C.POINTER(d)]
    L.lasto_net_train_step.restype = i
    L.lasto_learned_guess.argtypes = [P, P, P, P, P, C.POINTER(i)]
    L.lasto_learned_guess.restype = i
    L.lasto_learned_correction.argtypes = [P, P, P, P, P, C.POINTER(i)]
    L.lasto_learned_correction.restype = i
    L.lasto_net_correction_features.argtypes = [P, P, P, P, P, C.POINTER(d)]
    L.lasto_net_correction_features.restype = i
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != OK and status not in allow:
        raise LastoError(status, load().lasto_last_error().decode())
    return status


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype=None) -> int:
    """Device pointer of a contiguous CUDA/HIP tensor (float64 unless dtype is given)."""
    import torch
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError("expected a contiguous %s device tensor" % dtype)
    return t.data_ptr()


def status_string(s: int) -> str:
    return load().lasto_status_string(s).decode()


def mesh_graded_1d(lo, hi, n, planes, hmin, hmax, gmax=1.2, hmin_step=0.0):
    """Graded 1-D coordinates (host). Returns (x, g, hmin_used)."""
    pl = np.ascontiguousarray(planes, dtype=np.float64).ravel()
    x = np.zeros(n)
    g = np.zeros(1)
    hm = np.zeros(1)
    _check(load().lasto_mesh_graded_1d(lo, hi, n, _np_ptr(pl) if len(pl) else None, len(pl), hmin, hmax, gmax,
                                       hmin_step, _np_ptr(x), _np_ptr(g), _np_ptr(hm)))
    return x, float(g[0]), float(hm[0])


def mesh_for(axes) -> List[np.ndarray]:
    return [mesh_graded_1d(a.lo, a.hi, a.n, a.planes, a.hmin, a.hmax, a.gmax, a.hmin_step)[0] for a in axes]


def fdm_axis(x):
    """Host decomposition of the 1-D interior operator: (lam, S, Sinv) with
    A = S diag(lam) Sinv."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = len(x) - 2
    lam = np.zeros(m)
    S = np.zeros((m, m))
    Si = np.zeros((m, m))
    _check(load().lasto_fdm_axis(_np_ptr(x), len(x), _np_ptr(lam), _np_ptr(S), _np_ptr(Si)))
    return lam, S, Si


def make_atoms(atoms: Sequence) -> C.Array:
    """lasto_atom array from objects with the fields of inputs.Atom."""
    arr = (Atom * max(len(atoms), 1))()
    for k, a in enumerate(atoms):
        A = arr[k]
        for c in range(3):
            A.center[c] = float(a.center[c])
        A.radius = float(a.radius)
        A.q = float(a.q)
        A.kind = int(a.kind)
        A.lmax = int(a.lmax)
        A.width = float(a.width)
        A.rho_R = float(a.rho_R)
        A.drho_R = float(a.drho_R)
        A.alpha = float(a.alpha)
        for c, v in enumerate(np.asarray(a.clm, dtype=np.float64).ravel()[:24]):
            A.clm[c] = float(v)
    return arr


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load().lasto_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Grid:
    """A tensor-product grid with its multigrid hierarchy on the current device."""

    def __init__(self, x, y, z, n_batch: int = 1, stream=None):
        import torch
        self.coords = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z)]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        h = C.c_void_p()
        xs, ys, zs = self.coords
        _check(load().lasto_grid_create(_np_ptr(xs), len(xs), _np_ptr(ys), len(ys), _np_ptr(zs), len(zs),
                                        n_batch, C.c_void_p(sp), C.byref(h)))
        self.h = h
        self.n_batch = n_batch
        self.copy_shape = (len(zs), len(ys), len(xs))
        self.shape = self.copy_shape if n_batch == 1 else (n_batch,) + self.copy_shape

    def close(self):
        if getattr(self, "h", None):
            load().lasto_grid_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone; the process
        # releases the device memory itself
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def levels(self) -> List[tuple]:
        n = C.c_int()
        _check(load().lasto_grid_levels(self.h, C.byref(n)))
        out = []
        for l in range(n.value):
            s = np.zeros(3, dtype=np.int32)
            _check(load().lasto_grid_level_shape(self.h, l, _np_ptr(s)))
            out.append(tuple(int(v) for v in s))
        return out

    def level_nodes(self, level: int):
        """Finest-level indices of level `level`'s nodes per axis: (ix, iy, iz)."""
        nx, ny, nz = self.levels()[level]
        out = [np.zeros(n, dtype=np.int32) for n in (nx, ny, nz)]
        _check(load().lasto_grid_level_nodes(self.h, level, *[_np_ptr(a) for a in out]))
        return tuple(out)

    def empty(self):
        import torch
        return torch.zeros(self.shape, dtype=torch.float64, device="cuda")

    def _atom_table(self, atoms):
        """A flat atom table: one list per right-hand side for a batch (equal lengths)."""
        if self.n_batch == 1:
            return make_atoms(atoms), len(atoms)
        if len(atoms) != self.n_batch or len({len(a) for a in atoms}) != 1:
            raise ValueError("a batched grid needs one atom list per right-hand side, all of one length")
        return make_atoms([a for lst in atoms for a in lst]), len(atoms[0])

    def pseudo_density(self, atoms, rho_out=None, rho_interstitial=None, renormalize=True, moments=False):
        arr, na = self._atom_table(atoms)
        if rho_out is None:
            rho_out = self.empty()
        Q = np.zeros((self.n_batch, 25))
        _check(load().lasto_pseudo_density(self.h, na, C.cast(arr, C.c_void_p),
                                           None if rho_interstitial is None else _dev_ptr(rho_interstitial),
                                           int(renormalize), _dev_ptr(rho_out), _np_ptr(Q) if moments else None))
        if self.n_batch == 1:
            Q = Q[0]
        return (rho_out, Q) if moments else rho_out

    def poisson_solve(self, rho, v, allow_fail: bool = False, atoms=None, guess_net=None, coarse_net=None,
                      **opts):
        """lasto_poisson_solve. atoms (guess 2, 3): as for pseudo_density;
        guess_net, coarse_net: Net objects (or None)."""
        keep = None
        if atoms is not None:
            keep, na = self._atom_table(atoms)
            opts["n_atoms"] = na
            opts["atoms"] = C.cast(keep, C.c_void_p).value
        if guess_net is not None:
            opts["guess_net"] = guess_net.h.value
        if coarse_net is not None:
            opts["coarse_net"] = coarse_net.h.value
        o = default_opts(**opts)
        info = SolveInfo()
        st = load().lasto_poisson_solve(self.h, _dev_ptr(rho), _dev_ptr(v), C.byref(o), C.byref(info))
        d = info.as_dict()
        d["status"] = st
        if not allow_fail:
            _check(st)
        return d

    def sphere_interp(self, v, centers, radii, dirs=None, noalloc: bool = False) -> np.ndarray:
        """V at C_a + R_a d_k (lasto_sphere_interp; noalloc: lasto_sphere_interp_noalloc)."""
        centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        radii = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        na = len(centers)
        if dirs is None:
            nd = 64
            dp = None
        else:
            dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
            nd = len(dirs)
            dp = _np_ptr(dirs)
        out = np.zeros((self.n_batch, na, nd))
        fn = load().lasto_sphere_interp_noalloc if noalloc else load().lasto_sphere_interp
        _check(fn(self.h, _dev_ptr(v), na, _np_ptr(centers), _np_ptr(radii), nd, dp, _np_ptr(out)))
        return out[0] if self.n_batch == 1 else out

    def apply(self, u, Au=None):
        if Au is None:
            Au = self.empty()
        _check(load().lasto_apply(self.h, _dev_ptr(u), _dev_ptr(Au)))
        return Au

    def rb_sweep(self, u_in, rho, u_out=None, first_colour: int = 0):
        if u_out is None:
            u_out = u_in.clone()
        _check(load().lasto_rb_sweep(self.h, _dev_ptr(u_in), _dev_ptr(rho), _dev_ptr(u_out), first_colour))
        return u_out

    def smooth(self, level: int, f, u, nsweeps: int, first_colour: int = 0, zero_in: bool = False,
               fused: bool = True, precision: int = 0, dot: bool = False):
        """Red-black half-sweeps on A u = f (zero faces) at a level; u is updated in place.
        Returns the partial <f, u>_W of the last two half-sweeps when dot is set, else None."""
        d = C.c_double(0.0)
        _check(load().lasto_smooth(self.h, level, precision, _dev_ptr(f), _dev_ptr(u), nsweeps, first_colour,
                                   int(zero_in), int(fused), C.byref(d) if dot else None))
        return d.value if dot else None

    def boundary_values(self, rho, v, bc: int = 1, lmax_bc: int = 4):
        Q = np.zeros((self.n_batch, 25))
        _check(load().lasto_boundary_values(self.h, _dev_ptr(rho), bc, lmax_bc, _dev_ptr(v), _np_ptr(Q)))
        return Q[0] if self.n_batch == 1 else Q

    def analytic_guess(self, atoms, v):
        arr, na = self._atom_table(atoms)
        _check(load().lasto_analytic_guess(self.h, na, C.cast(arr, C.c_void_p), _dev_ptr(v)))
        return v

    def interstitial_density(self, centers, radii, shells, coef, occ, rho_out=None):
        """rho_out = sum_k f_k psi_k^2 at the nodes outside every sphere (zero
        inside); shells = [(n, l, zeta), ...] on every atom, coef a device
        [n_basis][n_occ] float64 tensor, occ host [n_occ]. One copy of the grid."""
        import torch
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        r = None if radii is None else np.ascontiguousarray(radii, dtype=np.float64).ravel()
        sh = (Shell * len(shells))()
        for k, (n, l, z) in enumerate(shells):
            sh[k].n, sh[k].l, sh[k].zeta = int(n), int(l), float(z)
        f = np.ascontiguousarray(occ, dtype=np.float64).ravel()
        if rho_out is None:
            rho_out = torch.empty(self.copy_shape, dtype=torch.float64, device="cuda")
        _check(load().lasto_interstitial_density(self.h, len(c), _np_ptr(c), None if r is None else _np_ptr(r),
                                                 len(shells), C.cast(sh, C.c_void_p), len(f), _dev_ptr(coef),
                                                 _np_ptr(f), _dev_ptr(rho_out)))
        return rho_out

    def fdm_solve(self, rho, v, bc: int = 1, lmax_bc: int = 4) -> dict:
        """Direct solve by fast diagonalisation (v's faces set, interior
        overwritten); returns the solve info as a dict."""
        info = SolveInfo()
        _check(load().lasto_fdm_solve(self.h, _dev_ptr(rho), _dev_ptr(v), bc, lmax_bc, C.byref(info)))
        return info.as_dict()

    def matrix_elements(self, v, centers, radii, shells):
        """Interstitial S and H (device [n_basis][n_basis] float64 tensors) by
        grid quadrature at the nodes outside every sphere, potential v."""
        import torch
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        sh = (Shell * len(shells))()
        for k, (n, l, z) in enumerate(shells):
            sh[k].n, sh[k].l, sh[k].zeta = int(n), int(l), float(z)
        nb = len(c) * sum(2 * int(l) + 1 for _, l, _ in shells)
        S = torch.empty((nb, nb), dtype=torch.float64, device="cuda")
        H = torch.empty((nb, nb), dtype=torch.float64, device="cuda")
        _check(load().lasto_matrix_elements(self.h, _dev_ptr(v), len(c), _np_ptr(c), _np_ptr(r), len(shells),
                                            C.cast(sh, C.c_void_p), _dev_ptr(S), _dev_ptr(H)))
        return S, H

    def learned_guess(self, net: "Net", rho, v):
        return _learned_call(load().lasto_learned_guess, self, net, rho, v)

    def learned_correction(self, net: "Net", rho, v):
        return _learned_call(load().lasto_learned_correction, self, net, rho, v)


class Spheres:
    """A set of muffin-tin spheres on a grid: projection of V onto y_LM on
    each boundary (eq. (3.6)), the interior radial solve (eq. (3.4)) and the
    energy integral of V rho (Section 4). Arrays carry a leading batch
    dimension on a batched grid."""

    def __init__(self, grid: Grid, centers, radii, Z=None, n_theta: int = 8, n_phi: int = 9, n_rad: int = 429,
                 r_min: float = 1e-5):
        self.grid = grid
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        z = None if Z is None else np.ascontiguousarray(Z, dtype=np.float64).ravel()
        self.n_atoms, self.n_rad = len(c), n_rad
        h = C.c_void_p()
        _check(load().lasto_spheres_create(grid.h, len(c), _np_ptr(c), _np_ptr(r), None if z is None else _np_ptr(z),
                                           n_theta, n_phi, n_rad, r_min, C.byref(h)))
        self.h = h
        lead = () if grid.n_batch == 1 else (grid.n_batch,)
        self.vlm_R_shape = lead + (self.n_atoms, 25)
        self.radial_shape = lead + (self.n_atoms, 25, n_rad)

    def close(self):
        if getattr(self, "h", None):
            load().lasto_spheres_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone; the process
        # releases the device memory itself
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def density_terms(self, rho_lm, rho, lmin: int = 1):
        """rho += sum_(L >= lmin) rho_LM(r) y_LM inside each sphere (in place)."""
        _check(load().lasto_sphere_density_terms(self.h, _dev_ptr(rho_lm), lmin, _dev_ptr(rho)))
        return rho

    def project(self, v, vlm_R=None):
        import torch
        if vlm_R is None:
            vlm_R = torch.empty(self.vlm_R_shape, dtype=torch.float64, device="cuda")
        _check(load().lasto_sphere_project(self.h, _dev_ptr(v), _dev_ptr(vlm_R)))
        return vlm_R

    def radial(self, vlm_R, rho_lm, v_lm=None):
        import torch
        if v_lm is None:
            v_lm = torch.empty(self.radial_shape, dtype=torch.float64, device="cuda")
        _check(load().lasto_sphere_radial(self.h, _dev_ptr(vlm_R), _dev_ptr(rho_lm), _dev_ptr(v_lm)))
        return v_lm

    def energy(self, v, rho, v_lm, rho_lm) -> np.ndarray:
        """[grid part, sphere part] of int V rho dV ([n_batch][2] for a batch)."""
        e = np.zeros((self.grid.n_batch, 2))
        _check(load().lasto_sphere_energy(self.h, _dev_ptr(v), _dev_ptr(rho), _dev_ptr(v_lm), _dev_ptr(rho_lm),
                                          _np_ptr(e)))
        return e[0] if self.grid.n_batch == 1 else e


def _learned_call(fn, grid, net, rho, v):
    rel = np.zeros(2 * grid.n_batch)
    acc = C.c_int()
    _check(fn(grid.h, net.h, _dev_ptr(rho), _dev_ptr(v), _np_ptr(rel), C.byref(acc)))
    if grid.n_batch == 1:
        return dict(rel_before=float(rel[0]), rel_after=float(rel[1]), accepted=bool(acc.value))
    return dict(rel_before=rel[0::2].tolist(), rel_after=rel[1::2].tolist(), accepted=int(acc.value))


class Net:
    """The learned-guess U-Net (weights, Adam state and activations on the device)."""

    def __init__(self, shape, ch=(16, 32, 48, 64), seed=1, rho_scale=0.1, pot_scale=0.01, h_ref=0.25,
                 out_scale=1.0, stream=None):
        import torch
        nz, ny, nx = shape
        cfg = NetConfig()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        for k in range(4):
            cfg.ch[k] = ch[k]
        cfg.seed = seed
        cfg.rho_scale, cfg.pot_scale, cfg.h_ref, cfg.out_scale = rho_scale, pot_scale, h_ref, out_scale
        self.cfg = cfg
        self.shape = (nz, ny, nx)
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        h = C.c_void_p()
        _check(load().lasto_net_create(C.byref(cfg), C.c_void_p(sp), C.byref(h)))
        self.h = h
        n = C.c_longlong()
        _check(load().lasto_net_param_count(h, C.byref(n)))
        self.nparam = n.value

    def save(self, path: str):
        """Checkpoint: masters, Adam moments and step, seed and scales (lasto_net_save)."""
        _check(load().lasto_net_save(self.h, os.fsencode(path)))

    def load_checkpoint(self, path: str):
        """Resume from a checkpoint (lasto_net_load); the grid size stays this net's."""
        _check(load().lasto_net_load(self.h, os.fsencode(path)))
        _check(load().lasto_net_get_config(self.h, C.byref(self.cfg), None))

    def coarse_pair(self, grid: "Grid", rho, v, level: int, nu1: int = 2):
        """Training pair of the learned coarse correction at `level` for iterate v:
        (features x, target t, residual scale s, level shape (nz, ny, nx))."""
        import torch
        nz, ny, nx = grid.levels()[level][::-1]
        x = torch.zeros((nz, ny, nx, 8), dtype=torch.int16, device="cuda")
        t = torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda")
        s = C.c_double()
        dims = np.zeros(3, dtype=np.int32)
        _check(load().lasto_coarse_pair(grid.h, self.h, _dev_ptr(rho), _dev_ptr(v), level, nu1,
                                        _dev_ptr(x, torch.int16), _dev_ptr(t, torch.float32), C.byref(s),
                                        _np_ptr(dims)))
        return x, t, s.value, (nz, ny, nx)

    def set_grid(self, shape):
        """Run on a grid of shape (nz, ny, nx), at most the creation size per axis."""
        nz, ny, nx = shape
        _check(load().lasto_net_set_grid(self.h, nx, ny, nz))
        self.shape = (nz, ny, nx)

    # stored tensors (lasto_net_tensor), in header order
    TENSORS = ["e0", "e1", "e2", "e3", "m3", "d2", "d1", "d0", "u2", "u1", "u0",
               "g0", "g1", "g2", "g3", "g4", "g5", "g6", "g7", "du0", "du1", "du2"]

    def tensor(self, name: str):
        """A stored BF16 tensor as int16 bit patterns on the device, [nz][ny][nx][c]."""
        import torch
        which = self.TENSORS.index(name)
        dims = np.zeros(4, dtype=np.int32)
        _check(load().lasto_net_tensor(self.h, which, None, 0, _np_ptr(dims)))
        nx, ny, nz, c = (int(d) for d in dims)
        out = torch.empty((nz, ny, nx, c), dtype=torch.int16, device="cuda")
        _check(load().lasto_net_tensor(self.h, which, _dev_ptr(out, torch.int16), out.numel(), _np_ptr(dims)))
        return out

    def adam_steps(self) -> int:
        cfg, st = NetConfig(), C.c_longlong()
        _check(load().lasto_net_get_config(self.h, C.byref(cfg), C.byref(st)))
        return st.value

    def close(self):
        if getattr(self, "h", None):
            load().lasto_net_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone; the process
        # releases the device memory itself
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        a = np.zeros(self.nparam, dtype=np.float32)
        _check(load().lasto_net_get_params(self.h, _np_ptr(a), self.nparam))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        _check(load().lasto_net_set_params(self.h, _np_ptr(a), self.nparam))

    def grads(self) -> np.ndarray:
        a = np.zeros(self.nparam, dtype=np.float32)
        _check(load().lasto_net_get_grads(self.h, _np_ptr(a), self.nparam))
        return a

    def features(self, grid: Grid, rho, v, x=None):
        """BF16 features as an int16 tensor [nz, ny, nx, 8] (bit patterns)."""
        import torch
        if x is None:
            x = torch.zeros(self.shape + (8,), dtype=torch.int16, device="cuda")
        _check(load().lasto_net_features(grid.h, self.h, _dev_ptr(rho), _dev_ptr(v), _dev_ptr(x, torch.int16)))
        return x

    def correction_features(self, grid: Grid, rho, v, x=None):
        """(features of iterate v for the correction net, residual RMS s)"""
        import torch
        if x is None:
            x = torch.zeros(self.shape + (8,), dtype=torch.int16, device="cuda")
        s = C.c_double()
        _check(load().lasto_net_correction_features(grid.h, self.h, _dev_ptr(rho), _dev_ptr(v),
                                                    _dev_ptr(x, torch.int16), C.byref(s)))
        return x, s.value

    def forward(self, x, y=None):
        import torch
        if y is None:
            y = torch.zeros(self.shape, dtype=torch.float32, device="cuda")
        _check(load().lasto_net_forward(self.h, _dev_ptr(x, torch.int16), _dev_ptr(y, torch.float32)))
        return y

    def backward(self, x, target, weight) -> float:
        import torch
        loss = C.c_double()
        _check(load().lasto_net_backward(self.h, _dev_ptr(x, torch.int16), _dev_ptr(target, torch.float32),
                                         _dev_ptr(weight, torch.float32), C.byref(loss)))
        return loss.value

    def adam_step(self, lr: float):
        _check(load().lasto_net_adam_step(self.h, lr))

    def train_step(self, x, target, weight, lr: float) -> float:
        import torch
        loss = C.c_double()
        _check(load().lasto_net_train_step(self.h, _dev_ptr(x, torch.int16), _dev_ptr(target, torch.float32),
                                           _dev_ptr(weight, torch.float32), lr, C.byref(loss)))
        return loss.value


def hartree_step(grid: Grid, atoms, rtol=1e-10, dirs=None, **opts):
    """The whole path on the GPU: pseudo-density -> Poisson solve with
    multipole faces -> values on the sphere boundaries."""
    rho = grid.pseudo_density(atoms)
    v = grid.empty()
    info = grid.poisson_solve(rho, v, rtol=rtol, **opts)
    centers = np.array([a.center for a in atoms])
    radii = np.array([a.radius for a in atoms])
    sph = grid.sphere_interp(v, centers, radii, dirs)
    return dict(rho=rho, v=v, info=info, sphere=sph)


def stream_probe(a, dst, b=None, stream=None):
    """dst = a (or a + b) by the library's streaming probe on the current stream."""
    import torch
    st = stream or torch.cuda.current_stream()
    _check(load().lasto_stream_probe(_dev_ptr(a), None if b is None else _dev_ptr(b), _dev_ptr(dst),
                                     a.numel() * 8, C.c_void_p(st.cuda_stream)))
