"""ColaSim: PyTorch-facing wrapper of a libcola context.

PyTorch provides the device memory (the workspace and the in/out tensors)
and the HIP stream; every computation runs in libcola's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, cola_params, dptr


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous(), "device tensor must be contiguous"
    return C.c_void_p(t.data_ptr())


def make_params(np_side, nmesh, box, omega_m=0.27, n_lpt=-2.5, a_init=0.02, flags=0):
    lib = _lib.load()
    p = cola_params()
    lib.cola_params_default(C.byref(p), np_side, nmesh, box)
    p.omega_m, p.n_lpt, p.a_init, p.flags = omega_m, n_lpt, a_init, flags
    return p


class ColaSim:
    """One COLA realisation on one GPU.

    Particle arrays are (3, np^3) float32 in mesh-cell units; meshes are
    (nmesh, nmesh, nmesh) float32, C order.
    """

    def __init__(self, np_side, nmesh, box, omega_m=0.27, n_lpt=-2.5, a_init=0.02,
                 flags=0, device="cuda", stream=None):
        self.lib = _lib.load()
        self._owned = True
        p = make_params(np_side, nmesh, box, omega_m, n_lpt, a_init, flags)
        self.params = p
        nbytes = C.c_size_t()
        check(self.lib.cola_workspace_query(C.byref(p), C.byref(nbytes)), what="workspace_query")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        check(self.lib.cola_create(C.byref(p), _ptr(self.workspace), nbytes.value,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx)),
              what="create")
        self.ctx = ctx
        self.np_side, self.nmesh, self.box = np_side, nmesh, box
        self.n_particles = np_side ** 3

    @classmethod
    def _view(cls, lib, ctx, params, device, stream, owner):
        """A context owned by a batch (not destroyed by close())."""
        self = cls.__new__(cls)
        self.lib, self.ctx, self.params = lib, C.c_void_p(ctx), params
        self._owned = False
        self._owner = owner
        self.device, self.stream = device, stream
        self.np_side, self.nmesh, self.box = params.np, params.nmesh, params.box
        self.n_particles = params.np ** 3
        return self

    def close(self):
        if self.ctx and self._owned:
            self.lib.cola_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _chk(self, code, what):
        return check(code, self.ctx, what)

    def particles(self):
        return torch.empty((3, self.n_particles), dtype=torch.float32, device=self.device)

    # -- initial conditions ------------------------------------------------
    def init_from_noise(self, noise: torch.Tensor, k, pk):
        k = np.ascontiguousarray(k, np.float64)
        pk = np.ascontiguousarray(pk, np.float64)
        self._chk(self.lib.cola_init_2lpt_from_noise(self.ctx, _ptr(noise), dptr(k), dptr(pk), len(k)),
                  "init_2lpt_from_noise")

    def init_2lpt(self, seed: int, k, pk):
        k = np.ascontiguousarray(k, np.float64)
        pk = np.ascontiguousarray(pk, np.float64)
        self._chk(self.lib.cola_init_2lpt(self.ctx, seed, dptr(k), dptr(pk), len(k), self.box,
                                          self.np_side), "init_2lpt")

    def noise(self, seed: int) -> torch.Tensor:
        out = torch.empty((self.np_side,) * 3, dtype=torch.float32, device=self.device)
        self._chk(self.lib.cola_noise(self.ctx, seed, _ptr(out)), "noise")
        return out

    # -- stepping and outputs ----------------------------------------------
    def step(self, a0: float, a1: float):
        self._chk(self.lib.cola_step(self.ctx, a0, a1), "step")

    def run(self, edges):
        for a0, a1 in zip(edges[:-1], edges[1:]):
            self.step(a0, a1)

    def density(self, out=None, disp=None) -> torch.Tensor:
        """Density contrast of the current positions, or of the displacement
        field ``disp`` (3 x np^3, mesh units) on the same particle lattice."""
        if out is None:
            out = torch.empty((self.nmesh,) * 3, dtype=torch.float32, device=self.device)
        if disp is None:
            self._chk(self.lib.cola_density(self.ctx, _ptr(out)), "density")
        else:
            self._chk(self.lib.cola_density_of(self.ctx, _ptr(disp), _ptr(out)), "density_of")
        return out

    def force(self, out=None) -> torch.Tensor:
        if out is None:
            out = self.particles()
        self._chk(self.lib.cola_force(self.ctx, _ptr(out)), "force")
        return out

    def pm_gradient(self, a: float, delta: torch.Tensor, comps=(0, 1, 2)):
        """Force meshes g_d (mesh units) of the density contrast ``delta``
        (nmesh^3) at scale factor a; returns {d: (nmesh,)*3 tensor} for d in comps."""
        out = {d: torch.empty((self.nmesh,) * 3, dtype=torch.float32, device=self.device) for d in comps}
        ptrs = [_ptr(out[d]) if d in out else None for d in range(3)]
        self._chk(self.lib.cola_pm_gradient(self.ctx, float(a), _ptr(delta), *ptrs), "pm_gradient")
        return out

    def velocity(self, out=None, rsd_axis=None, sdisp=None):
        """Canonical particle velocity at the position time a_x (3 x np^3, mesh
        units); with rsd_axis also the redshift-space displacement along that
        axis.  Returns out, or (out, sdisp) when rsd_axis is given."""
        if out is None:
            out = self.particles()
        if rsd_axis is not None and sdisp is None:
            sdisp = self.particles()
        self._chk(self.lib.cola_velocity(self.ctx, _ptr(out), _ptr(sdisp) if rsd_axis is not None else None,
                                         -1 if rsd_axis is None else int(rsd_axis)), "velocity")
        return out if rsd_axis is None else (out, sdisp)

    def snapshot(self, a1: float, a_s: float, rsd_axis=None):
        """Displacement and canonical velocity at a_s inside the coming step
        a_x -> a1 (state unchanged); with rsd_axis also the redshift-space
        displacement.  Returns (disp, vel) or (disp, vel, sdisp)."""
        d, v = self.particles(), self.particles()
        sd = self.particles() if rsd_axis is not None else None
        self._chk(self.lib.cola_snapshot(self.ctx, a1, a_s, _ptr(d), _ptr(v), _ptr(sd) if sd is not None else None,
                                         -1 if rsd_axis is None else int(rsd_axis)), "snapshot")
        return (d, v) if sd is None else (d, v, sd)

    def fof(self, b_frac=0.2, out=None):
        """Friends-of-friends labels (np^3 int32: smallest id of each particle's group)."""
        n = C.c_size_t()
        self._chk(self.lib.cola_fof_workspace_bytes(self.ctx, C.byref(n)), "fof_workspace_bytes")
        work = torch.empty((n.value + 255) // 4 + 64, dtype=torch.int32, device=self.device)
        off = (-work.data_ptr()) % 256
        wptr = C.c_void_p(work.data_ptr() + off)
        if out is None:
            out = torch.empty(self.n_particles, dtype=torch.int32, device=self.device)
        self._chk(self.lib.cola_fof(self.ctx, float(b_frac), _ptr(out), wptr, n.value), "fof")
        return out

    def fof_halos(self, labels, vel=None, min_members=32, max_halos=None):
        """Halo catalogue of FoF labels: dict of root, count (int32), pos and
        (with vel) vel, (3, n) float32 in mesh units, in increasing root id."""
        n = C.c_size_t()
        self._chk(self.lib.cola_fof_halos_workspace_bytes(self.ctx, int(min_members), C.byref(n)),
                  "fof_halos_workspace_bytes")
        work = torch.empty((n.value + 255) // 4 + 64, dtype=torch.int32, device=self.device)
        wptr = C.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        cap = int(max_halos) if max_halos is not None else self.n_particles // int(min_members) + 1
        root = torch.empty(cap, dtype=torch.int32, device=self.device)
        cnt = torch.empty(cap, dtype=torch.int32, device=self.device)
        pos = torch.empty((3, cap), dtype=torch.float32, device=self.device)
        hv = torch.empty((3, cap), dtype=torch.float32, device=self.device) if vel is not None else None
        nh = C.c_int32()
        self._chk(self.lib.cola_fof_halos(self.ctx, _ptr(labels), _ptr(vel) if vel is not None else None,
                                          int(min_members), cap, C.byref(nh), _ptr(root), _ptr(cnt), _ptr(pos),
                                          _ptr(hv) if hv is not None else None, wptr, n.value), "fof_halos")
        k = nh.value
        out = {"root": root[:k], "count": cnt[:k], "pos": pos[:, :k]}
        if hv is not None:
            out["vel"] = hv[:, :k]
        return out

    def pk_velocity(self, edges, axis=2):
        """Density and line-of-sight momentum spectra on the PM mesh:
        (kmean, P_dd, P_du, P_uu, counts)."""
        edges = np.ascontiguousarray(edges, np.float64)
        nb = len(edges) - 1
        out = [np.zeros(nb) for _ in range(4)]
        cnt = np.zeros(nb, np.int64)
        self._chk(self.lib.cola_pk_velocity(self.ctx, int(axis), dptr(edges), nb, *[dptr(o) for o in out],
                                            cnt.ctypes.data_as(C.POINTER(C.c_int64))), "pk_velocity")
        return (*out, cnt)

    def pk(self, edges, ngrid=None, disp=None, jing=False):
        """Binned P(k) of the current positions, or of the displacement field
        ``disp`` (3 x np^3, mesh units) on the same particle lattice.  jing:
        the smoothing and aliasing correction of Jing (2005) instead of the
        plain window division (current positions only)."""
        edges = np.ascontiguousarray(edges, np.float64)
        nb = len(edges) - 1
        km, p = np.zeros(nb), np.zeros(nb)
        nm = np.zeros(nb, np.int64)
        cnt = nm.ctypes.data_as(C.POINTER(C.c_int64))
        if jing:
            if disp is not None:
                raise ValueError("the Jing-corrected spectrum is of the current positions")
            self._chk(self.lib.cola_pk_jing(self.ctx, ngrid or self.nmesh, dptr(edges), nb, dptr(km), dptr(p),
                                            cnt), "pk_jing")
        elif disp is None:
            self._chk(self.lib.cola_pk(self.ctx, ngrid or self.nmesh, dptr(edges), nb, dptr(km), dptr(p), cnt),
                      "pk")
        else:
            self._chk(self.lib.cola_pk_of(self.ctx, _ptr(disp), ngrid or self.nmesh, dptr(edges), nb, dptr(km),
                                          dptr(p), cnt), "pk_of")
        return km, p, nm

    def get_state(self, which=("disp", "vres", "psi1", "psi2"), out=None):
        """Copies of the named state arrays (new tensors, or the ones in ``out``)
        and the times a_x, a_v."""
        names = ("disp", "vres", "psi1", "psi2")
        out = dict(out or {})
        for n in which:
            if n not in out:
                out[n] = self.particles()
        ptrs = [_ptr(out[n]) if n in which else None for n in names]
        ax, av = C.c_double(), C.c_double()
        self._chk(self.lib.cola_get_state(self.ctx, *ptrs, C.byref(ax), C.byref(av)), "get_state")
        res = {n: out[n] for n in which}
        res.update(a_x=ax.value, a_v=av.value)
        return res

    def set_state(self, disp, vres, psi1, psi2, a_x, a_v):
        """Arrays given as None keep the context's (every array on the first call)."""
        p = [None if t is None else _ptr(t) for t in (disp, vres, psi1, psi2)]
        self._chk(self.lib.cola_set_state(self.ctx, *p, a_x, a_v), "set_state")

    def fft3d(self, mesh: torch.Tensor, n: int, inverse=False):
        self._chk(self.lib.cola_fft3d(self.ctx, n, _ptr(mesh), int(inverse)), "fft3d")

    # -- adjoint (reverse mode) -------------------------------------------
    def step_adjoint(self, a0, a1, a_v0, disp0, dbar, vbar, psi1bar, psi2bar, slot=None):
        """Cotangents (dbar, vbar) at a1 -> at a0 in place; psi bars accumulate.
        slot: the force slot step_keep filled for this step (forces read, not
        recomputed)."""
        if slot is None:
            self._chk(self.lib.cola_step_adjoint(self.ctx, a0, a1, a_v0, _ptr(disp0), _ptr(dbar), _ptr(vbar),
                                                 _ptr(psi1bar), _ptr(psi2bar)), "step_adjoint")
        else:
            self._chk(self.lib.cola_step_adjoint_kept(self.ctx, a0, a1, a_v0, _ptr(disp0), _ptr(slot),
                                                      _ptr(dbar), _ptr(vbar), _ptr(psi1bar), _ptr(psi2bar)),
                      "step_adjoint_kept")

    def force_slot(self) -> torch.Tensor:
        """A device buffer for step_keep (the three force meshes of one step)."""
        n = C.c_size_t()
        self._chk(self.lib.cola_force_slot_bytes(self.ctx, C.byref(n)), "force_slot_bytes")
        return torch.empty(n.value // 4, dtype=torch.float32, device=self.device)

    def step_keep(self, a0: float, a1: float, slot: torch.Tensor):
        """step(a0, a1), leaving the step's force meshes in slot."""
        self._chk(self.lib.cola_step_keep(self.ctx, a0, a1, _ptr(slot)), "step_keep")

    def density_adjoint(self, disp, delta_bar, dbar):
        """dbar += d<delta_bar, density(disp)>/d disp."""
        self._chk(self.lib.cola_density_adjoint(self.ctx, _ptr(disp), _ptr(delta_bar), _ptr(dbar)),
                  "density_adjoint")

    def pk_adjoint(self, disp, edges, cbar, dbar, ngrid=None):
        """dbar += d(sum_b cbar_b P_b)/d disp."""
        edges = np.ascontiguousarray(edges, np.float64)
        cbar = np.ascontiguousarray(cbar, np.float64)
        self._chk(self.lib.cola_pk_adjoint(self.ctx, _ptr(disp), ngrid or self.nmesh, dptr(edges),
                                           len(edges) - 1, dptr(cbar), _ptr(dbar)), "pk_adjoint")

    def init_adjoint(self, noise, dbar0, psi1bar, psi2bar):
        out = torch.empty_like(noise)
        self._chk(self.lib.cola_init_2lpt_adjoint(self.ctx, _ptr(noise), _ptr(dbar0), _ptr(psi1bar),
                                                  _ptr(psi2bar), _ptr(out)), "init_2lpt_adjoint")
        return out

    def stage_times(self):
        """Per-stage (ms total, launches) since the last call (needs COLA_F_STAGE_TIMERS)."""
        ms = np.zeros(len(_lib.STAGES))
        cnt = np.zeros(len(_lib.STAGES), np.int64)
        self._chk(self.lib.cola_stage_times(self.ctx, dptr(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64))),
                  "stage_times")
        return {n: (float(m), int(k)) for n, m, k in zip(_lib.STAGES, ms, cnt)}

    def synchronize(self):
        self._chk(self.lib.cola_synchronize(self.ctx), "synchronize")

    def autotune(self, reps=3):
        """Times the column-pass block orders of the PM step at this mesh
        length and keeps the fastest (process-wide).  Returns
        ({pass kind: order}, {(pass kind, order): ms})."""
        best = (C.c_int32 * 3)()
        ms = np.zeros(6)
        self._chk(self.lib.cola_autotune(self.ctx, int(reps), best, dptr(ms)), "autotune")
        kinds = ("plain", "green", "grad")
        return ({kinds[k]: int(best[k]) for k in range(3)},
                {(kinds[k], o): float(ms[2 * k + o]) for k in range(3) for o in (0, 1)})


def fft_schedule(n, pass_kind, order=None):
    """Get (and with order, set) the column-pass block order (1: contiguous
    block ranges per XCD, 0: round-robin) of pass kind pass_kind
    (_lib.PASS_PLAIN / PASS_GREEN / PASS_GRAD) at transform length n;
    returns the value in force before the call."""
    lib = _lib.load()
    cur = C.c_int32()
    check(lib.cola_fft_get_schedule(int(n), int(pass_kind), C.byref(cur)), what="fft_get_schedule")
    if order is not None:
        check(lib.cola_fft_set_schedule(int(n), int(pass_kind), int(order)), what="fft_set_schedule")
    return cur.value


class ColaBatch:
    """Many independent realisations stepped together (libcola batch).

    ``specs`` is a list of dicts with keys np, nmesh, box and optionally
    omega_m, n_lpt, a_init, flags.  ``mocks[i]`` is a ColaSim view of mock i
    for initial conditions, outputs and single steps.
    """

    def __init__(self, specs, device="cuda", stream=None, graph=True):
        self.lib = _lib.load()
        n = len(specs)
        arr = (cola_params * n)()
        for i, sp in enumerate(specs):
            arr[i] = make_params(sp["np"], sp["nmesh"], sp["box"], sp.get("omega_m", 0.27),
                                 sp.get("n_lpt", -2.5), sp.get("a_init", 0.02), sp.get("flags", 0))
        self.params = arr
        nbytes = C.c_size_t()
        check(self.lib.cola_batch_workspace_query(arr, n, C.byref(nbytes)), what="batch_workspace_query")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = C.c_void_p()
        check(self.lib.cola_batch_create(arr, n, _ptr(self.workspace), nbytes.value,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(b)),
              what="batch_create")
        self.batch = b
        self.mocks = [ColaSim._view(self.lib, self.lib.cola_batch_mock(b, i), arr[i], self.device,
                                    self.stream, self) for i in range(n)]
        self.set_graph(graph)

    def __len__(self):
        return len(self.mocks)

    @property
    def ngroups(self):
        return int(self.lib.cola_batch_ngroups(self.batch))

    def set_graph(self, enable: bool):
        check(self.lib.cola_batch_set_graph(self.batch, int(bool(enable))), what="batch_set_graph",
              batch=self.batch)

    def set_chunk_bytes(self, nbytes: int):
        check(self.lib.cola_batch_set_chunk_bytes(self.batch, int(nbytes)), what="batch_set_chunk_bytes",
              batch=self.batch)

    def step(self, a0: float, a1: float):
        check(self.lib.cola_batch_step(self.batch, a0, a1), what="batch_step", batch=self.batch)

    def run(self, edges):
        for a0, a1 in zip(edges[:-1], edges[1:]):
            self.step(a0, a1)

    def synchronize(self):
        check(self.lib.cola_batch_synchronize(self.batch), what="batch_synchronize", batch=self.batch)

    def close(self):
        if getattr(self, "batch", None):
            for m in self.mocks:
                m.ctx = None
            self.lib.cola_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def padded_cols(n: int) -> int:
    """Complex values per row of the padded in-place r2c mesh layout."""
    return ((n // 2 + 1) + 15) // 16 * 16


def step_scalars(np_side, nmesh, box, a_x, a_v, a1, omega_m=0.27, n_lpt=-2.5):
    lib = _lib.load()
    p = cola_params()
    lib.cola_params_default(C.byref(p), np_side, nmesh, box)
    p.omega_m, p.n_lpt = omega_m, n_lpt
    out = np.zeros(10)
    check(lib.cola_step_scalars(C.byref(p), a_x, a_v, a1, dptr(out)), what="step_scalars")
    return out
