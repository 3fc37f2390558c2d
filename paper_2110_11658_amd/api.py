"""Thin torch-facing wrapper of the libpbh C ABI (same entry points, tensors in).

All tensors must live on the context's GPU: positions/velocities float64
(n, 3) contiguous, masses float64 (n,). Calls enqueue on torch's current
stream. Neighbour lists come back as CSR (int64 offsets [n+1], int32 indices
in caller order); the order inside one list is unspecified.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (PBH_E_NBR_OVERFLOW, PBH_FP64, PBH_MIXED, PbhError, check, pbh_core_info, pbh_params,
                   pbh_stats)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, shape, name: str, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")


class Pbh:
    """One libpbh context (tree scratch lives on the GPU between calls)."""

    def __init__(self, device: int = 0, leaf_size: int = 8, n_crit: int = 0, key_bits: int = 0,
                 prec: str = "mixed", walk_tile: int = 0, lanes_per_particle: int = 0):
        self.L = _lib.load()
        self.device = device
        self.ctx = C.c_void_p()
        p = self._params(leaf_size, n_crit, key_bits, prec, walk_tile, lanes_per_particle)
        st = self.L.pbh_create(device, C.byref(p), C.byref(self.ctx))
        if st != 0:
            raise PbhError(st, self.L.pbh_status_string(st).decode())
        self.n = 0
        self.n_clusters = 0
        self._nbr_cap = 0
        self._built = (None, None)   # the tensors of the last build (pbh_force takes them again)

    @staticmethod
    def _params(leaf_size, n_crit, key_bits, prec, walk_tile=0, lanes_per_particle=0):
        pr = {"mixed": PBH_MIXED, "fp64": PBH_FP64}[prec]
        return pbh_params(int(leaf_size), int(n_crit), int(walk_tile), int(lanes_per_particle),
                          int(key_bits), pr)

    def set_params(self, leaf_size=8, n_crit=0, key_bits=0, prec="mixed", walk_tile=0,
                   lanes_per_particle=0):
        p = self._params(leaf_size, n_crit, key_bits, prec, walk_tile, lanes_per_particle)
        check(self.ctx, self.L.pbh_set_params(self.ctx, C.byref(p)))

    def params(self) -> dict:
        p = pbh_params()
        check(self.ctx, self.L.pbh_get_params(self.ctx, C.byref(p)))
        return {"leaf_size": p.leaf_size, "n_crit": p.n_crit, "walk_tile": p.walk_tile,
                "lanes_per_particle": p.lanes_per_particle, "key_bits": p.key_bits,
                "prec": "mixed" if p.prec == PBH_MIXED else "fp64"}

    def close(self):
        if self.ctx:
            self.L.pbh_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- pbh_build / pbh_build_batched ---------------------------------------
    def build(self, pos: torch.Tensor, mass: torch.Tensor):
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(mass, (n,), "mass")
        check(self.ctx, self.L.pbh_build(self.ctx, n, _ptr(pos), _ptr(mass), _stream()))
        self.n = n
        self.n_clusters = 1
        self._built = (pos, mass)

    def build_batched(self, offsets: Sequence[int], pos: torch.Tensor, mass: torch.Tensor):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        n = int(off[-1])
        _need(pos, (n, 3), "pos")
        _need(mass, (n,), "mass")
        check(self.ctx, self.L.pbh_build_batched(self.ctx, off.size - 1,
                                                 off.ctypes.data_as(C.c_void_p),
                                                 _ptr(pos), _ptr(mass), _stream()))
        self.n = n
        self.n_clusters = off.size - 1
        self._built = (pos, mass)

    # -- pbh_force / pbh_force_batched ---------------------------------------
    def _force(self, call, neighbours: bool, nbr_cap: Optional[int]):
        dev = torch.device("cuda", self.device)
        acc = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((self.n,), dtype=torch.float64, device=dev)
        if not neighbours:
            check(self.ctx, call(acc, pot, None, None, 0, None))
            return acc, pot, None, None
        off = torch.empty((self.n + 1,), dtype=torch.int64, device=dev)
        cap = int(nbr_cap if nbr_cap is not None else self._nbr_cap)
        for _ in range(2):
            idx = torch.empty((max(cap, 1),), dtype=torch.int32, device=dev)
            total = C.c_int64(0)
            st = call(acc, pot, off, idx, cap, C.byref(total))
            if st == PBH_E_NBR_OVERFLOW:
                cap = int(total.value * 1.25) + 1024
                continue
            check(self.ctx, st)
            self._nbr_cap = max(self._nbr_cap, cap)
            return acc, pot, off, idx[: total.value]
        raise PbhError(PBH_E_NBR_OVERFLOW, "neighbour capacity still too small")

    def force(self, r_in: float, r_out: float, theta: float, eps: float, neighbours: bool = True,
              nbr_cap: Optional[int] = None, r_buff: float = 0.0):
        """(acc [n,3], pot [n], nbr_off [n+1] | None, nbr_idx [total] | None).

        The lists hold every j with r_ij < r_out + r_buff (r_buff = 0: r_out)."""
        bp, bm = self._built

        def call(acc, pot, off, idx, cap, total):
            return self.L.pbh_force_buffered(self.ctx, _ptr(bp), _ptr(bm), float(r_in), float(r_out),
                                             float(r_buff), float(theta), float(eps), _ptr(acc),
                                             _ptr(pot), _ptr(off), _ptr(idx), int(cap), total,
                                             _stream())
        return self._force(call, neighbours, nbr_cap)

    def force_batched(self, r_in: Sequence[float], r_out: Sequence[float], theta: float, eps: float,
                      neighbours: bool = True, nbr_cap: Optional[int] = None,
                      r_buff: Optional[Sequence[float]] = None):
        ri = np.ascontiguousarray(np.asarray(r_in, dtype=np.float64))
        ro = np.ascontiguousarray(np.asarray(r_out, dtype=np.float64))
        if ri.size != self.n_clusters or ro.size != self.n_clusters:
            raise ValueError("need one r_in and r_out per cluster")
        rb = None
        if r_buff is not None:
            rb = np.ascontiguousarray(np.asarray(r_buff, dtype=np.float64))
            if rb.size != self.n_clusters:
                raise ValueError("need one r_buff per cluster")

        bp, bm = self._built

        def call(acc, pot, off, idx, cap, total):
            return self.L.pbh_force_batched_buffered(
                self.ctx, _ptr(bp), _ptr(bm), ri.ctypes.data_as(C.c_void_p),
                ro.ctypes.data_as(C.c_void_p),
                None if rb is None else rb.ctypes.data_as(C.c_void_p), float(theta), float(eps),
                _ptr(acc), _ptr(pot), _ptr(off), _ptr(idx), int(cap), total, _stream())
        return self._force(call, neighbours, nbr_cap)

    def force_into(self, r_in, r_out, theta, eps, acc: torch.Tensor, pot: torch.Tensor):
        """Forces into caller-owned tensors, no neighbour lists, no host wait."""
        _need(acc, (self.n, 3), "acc")
        _need(pot, (self.n,), "pot")
        bp, bm = self._built
        check(self.ctx, self.L.pbh_force(self.ctx, _ptr(bp), _ptr(bm), float(r_in), float(r_out),
                                         float(theta), float(eps), _ptr(acc), _ptr(pot), None, None,
                                         0, None, _stream()))

    # -- pbh_kdk --------------------------------------------------------------
    # -- pbh_irregular / pbh_irregular_batched -------------------------------
    def irregular(self, pos: torch.Tensor, vel: Optional[torch.Tensor], mass: torch.Tensor,
                  r_in, r_out, eps: float, nbr_off: torch.Tensor, nbr_idx: torch.Tensor,
                  targets: Optional[torch.Tensor] = None, jerk: bool = True, pot: bool = True,
                  validate: bool = True, batched: bool = False):
        """Irregular force, its time derivative and potential from neighbour
        lists (eq. fi, fidot, duncan). Returns (acc, jerk or None, pot or None),
        [n] rows in caller order, or one row per entry of ``targets``.
        ``validate`` waits and raises on out-of-range targets or list entries.
        With ``batched`` the radii are per-cluster sequences of the last
        batched build."""
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(mass, (n,), "mass")
        if jerk:
            _need(vel, (n, 3), "vel")
        _need(nbr_off, (n + 1,), "nbr_off", torch.int64)
        _need(nbr_idx, (nbr_idx.shape[0],), "nbr_idx", torch.int32)
        rows = n
        if targets is not None:
            _need(targets, (targets.shape[0],), "targets", torch.int32)
            rows = targets.shape[0]
        opts = dict(dtype=torch.float64, device=pos.device)
        acc = torch.empty((rows, 3), **opts)
        jk = torch.empty((rows, 3), **opts) if jerk else None
        ph = torch.empty((rows,), **opts) if pot else None
        if rows == 0:   # an empty target list (its data pointer would read as "all")
            return acc, jk, ph
        common = (float(eps), _ptr(nbr_off), _ptr(nbr_idx), int(nbr_idx.shape[0]),
                  int(rows if targets is not None else 0), _ptr(targets), _ptr(acc), _ptr(jk),
                  _ptr(ph), int(bool(validate)), _stream())
        if batched:
            if n != self.n:
                raise ValueError("batched irregular force needs the particles of the last build")
            ri = np.ascontiguousarray(r_in, dtype=np.float64)
            ro = np.ascontiguousarray(r_out, dtype=np.float64)
            if ri.shape != (self.n_clusters,) or ro.shape != (self.n_clusters,):
                raise ValueError("need one r_in and r_out per cluster")
            st = self.L.pbh_irregular_batched(self.ctx, _ptr(pos), _ptr(vel), _ptr(mass),
                                              ri.ctypes.data_as(C.c_void_p),
                                              ro.ctypes.data_as(C.c_void_p), *common)
        else:
            st = self.L.pbh_irregular(self.ctx, n, _ptr(pos), _ptr(vel), _ptr(mass), float(r_in),
                                      float(r_out), *common)
        check(self.ctx, st)
        return acc, jk, ph

    def irregular_noalloc(self, pos: torch.Tensor, vel: Optional[torch.Tensor], mass: torch.Tensor,
                          r_in: float, r_out: float, eps: float, nbr_off: torch.Tensor,
                          nbr_idx: torch.Tensor, acc: torch.Tensor, jerk: Optional[torch.Tensor],
                          pot: Optional[torch.Tensor], targets: Optional[torch.Tensor] = None,
                          validate: bool = True):
        """pbh_irregular_noalloc: as ``irregular`` into caller-given outputs
        (acc, and jerk/pot or None), with no device allocation by the library."""
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(mass, (n,), "mass")
        if jerk is not None:
            _need(vel, (n, 3), "vel")
        _need(nbr_off, (n + 1,), "nbr_off", torch.int64)
        _need(nbr_idx, (nbr_idx.shape[0],), "nbr_idx", torch.int32)
        rows = n
        if targets is not None:
            _need(targets, (targets.shape[0],), "targets", torch.int32)
            rows = targets.shape[0]
        _need(acc, (rows, 3), "acc")
        if jerk is not None:
            _need(jerk, (rows, 3), "jerk")
        if pot is not None:
            _need(pot, (rows,), "pot")
        if rows == 0:
            return
        st = self.L.pbh_irregular_noalloc(self.ctx, n, _ptr(pos), _ptr(vel), _ptr(mass),
                                          float(r_in), float(r_out), float(eps), _ptr(nbr_off),
                                          _ptr(nbr_idx), int(nbr_idx.shape[0]),
                                          int(rows if targets is not None else 0), _ptr(targets),
                                          _ptr(acc), _ptr(jerk), _ptr(pot), int(bool(validate)),
                                          _stream())
        check(self.ctx, st)

    # -- pbh_core -----------------------------------------------------------------
    def core(self, pos: torch.Tensor, mass: torch.Tensor, sample: torch.Tensor, eta: float = 0.02,
             densities: bool = True):
        """Core quantities from the 6 nearest neighbours of the sampled particles
        (int32 caller indices) of the last build: (rho [n_sample] or None, dict)."""
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(mass, (n,), "mass")
        _need(sample, (sample.shape[0],), "sample", torch.int32)
        rho = torch.empty(sample.shape[0], dtype=torch.float64, device=pos.device) if densities else None
        info = pbh_core_info()
        check(self.ctx, self.L.pbh_core(self.ctx, _ptr(pos), _ptr(mass), int(sample.shape[0]),
                                        _ptr(sample), float(eta), _ptr(rho), C.byref(info), _stream()))
        res = {"center": np.array(info.center[:]), "rho_core": info.rho_core, "r_core": info.r_core,
               "n_core": int(info.n_core), "r_half": info.r_half, "r_min": info.r_min,
               "dt_min": info.dt_min}
        return rho, res

    # -- pbh_hermite / pbh_p3t --------------------------------------------------
    def hermite(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                fr: Optional[torch.Tensor], r_in: float, r_out: float, eps: float,
                nbr_off: torch.Tensor, nbr_idx: torch.Tensor, dt_reg: float, eta: float = 0.02):
        """Integrate F_I with block Hermite steps over one regular step, in
        place (pos, vel). Returns dict(blocks, steps, kmax)."""
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(vel, (n, 3), "vel")
        _need(mass, (n,), "mass")
        if fr is not None:
            _need(fr, (n, 3), "fr")
        _need(nbr_off, (n + 1,), "nbr_off", torch.int64)
        st = np.zeros(3, dtype=np.int64)
        check(self.ctx, self.L.pbh_hermite(self.ctx, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(fr),
                                           float(r_in), float(r_out), float(eps), _ptr(nbr_off),
                                           _ptr(nbr_idx), int(nbr_idx.shape[0]), float(dt_reg),
                                           float(eta), st.ctypes.data_as(C.c_void_p), _stream()))
        return {"blocks": int(st[0]), "steps": int(st[1]), "kmax": int(st[2])}

    def p3t(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, r_in: float, r_out: float,
            r_buff: float, theta: float, eps: float, dt_reg: float, eta: float = 0.02, steps: int = 1):
        """P3T loop in place: per step kick, Hermite F_I over dt_reg, kick.
        Returns (energy [steps+1] on the device, dict(blocks, steps, kmax))."""
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(vel, (n, 3), "vel")
        _need(mass, (n,), "mass")
        energy = torch.empty(steps + 1, dtype=torch.float64, device=pos.device)
        st = np.zeros(3, dtype=np.int64)
        check(self.ctx, self.L.pbh_p3t(self.ctx, n, _ptr(pos), _ptr(vel), _ptr(mass), float(r_in),
                                       float(r_out), float(r_buff), float(theta), float(eps),
                                       float(dt_reg), float(eta), int(steps), _ptr(energy),
                                       st.ctypes.data_as(C.c_void_p), _stream()))
        self.n = n
        self.n_clusters = 1
        self._built = (pos, mass)
        return energy, {"blocks": int(st[0]), "steps": int(st[1]), "kmax": int(st[2])}

    def kdk(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, dt: float, steps: int,
            r_in: float, r_out: float, theta: float, eps: float, graph: bool = True,
            energy: Optional[torch.Tensor] = None) -> torch.Tensor:
        n = pos.shape[0]
        _need(pos, (n, 3), "pos")
        _need(vel, (n, 3), "vel")
        _need(mass, (n,), "mass")
        if energy is None:
            energy = torch.empty((steps + 1,), dtype=torch.float64, device=pos.device)
        _need(energy, (steps + 1,), "energy")
        fn = self.L.pbh_kdk_graph if graph else self.L.pbh_kdk_eager
        check(self.ctx, fn(self.ctx, n, _ptr(pos), _ptr(vel), _ptr(mass), float(dt), int(steps),
                           float(r_in), float(r_out), float(theta), float(eps), _ptr(energy),
                           _stream()))
        self.n = n
        self.n_clusters = 1
        self._built = (pos, mass)
        return energy

    # -- stats / debug ----------------------------------------------------------
    def set_timing(self, enable: bool = True):
        check(self.ctx, self.L.pbh_set_timing(self.ctx, int(bool(enable))))

    def stats(self) -> dict:
        s = pbh_stats()
        check(self.ctx, self.L.pbh_get_stats(self.ctx, C.byref(s)))
        out = {}
        for name, typ in pbh_stats._fields_:
            v = getattr(s, name)
            out[name] = float(v) if typ is C.c_double else int(v)
        return out

    def walk_clock_mhz(self) -> float:
        """Rate (MHz) of the device cycle counter during the last tree walk,
        from its workgroups' cycle and steady-clock counts (pbh_walk_clock)."""
        v = C.c_double(0.0)
        check(self.ctx, self.L.pbh_walk_clock(self.ctx, C.byref(v)))
        return float(v.value)

    def debug_series_log(self, x: torch.Tensor) -> torch.Tensor:
        """ln x by the logarithm of the irregular potential's Phi_R (device
        FP64 tensor of positive normal values)."""
        n = x.shape[0]
        _need(x, (n,), "x")
        y = torch.empty_like(x)
        check(self.ctx, self.L.pbh_debug_series_log(self.ctx, n, _ptr(x), _ptr(y), _stream()))
        return y

    def debug_herm_first_steps(self) -> np.ndarray:
        """First block step (ticks of dt_max / 2^40) of every particle in the
        last Hermite integration, caller order."""
        n = C.c_int64(0)
        check(self.ctx, self.L.pbh_debug_herm_first_steps(self.ctx, 0, None, C.byref(n)))
        t = np.zeros(n.value, dtype=np.int64)
        check(self.ctx, self.L.pbh_debug_herm_first_steps(self.ctx, n.value,
                                                          t.ctypes.data_as(C.c_void_p), C.byref(n)))
        return t

    def debug_groups(self):
        """(begin int32 [G], count int32 [G], box f64 [G,6]) of the last build."""
        ng = C.c_int64(0)
        check(self.ctx, self.L.pbh_debug_groups(self.ctx, 0, None, None, None, C.byref(ng)))
        b = np.zeros(ng.value, dtype=np.int32)
        c = np.zeros(ng.value, dtype=np.int32)
        box = np.zeros((ng.value, 6))
        check(self.ctx, self.L.pbh_debug_groups(self.ctx, ng.value, b.ctypes.data_as(C.c_void_p),
                                                c.ctypes.data_as(C.c_void_p),
                                                box.ctypes.data_as(C.c_void_p), C.byref(ng)))
        return b, c, box

    def debug_wave_log(self):
        """(walk [workgroups,2], nbr [workgroups,2]) of (groups, ticks at 100 MHz)."""
        nw, nn = C.c_int64(0), C.c_int64(0)
        check(self.ctx, self.L.pbh_debug_wave_log(self.ctx, None, None, 0, C.byref(nw), C.byref(nn)))
        cap = max(nw.value, nn.value)
        a = np.zeros((cap, 2), dtype=np.uint64)
        b = np.zeros((cap, 2), dtype=np.uint64)
        check(self.ctx, self.L.pbh_debug_wave_log(self.ctx, a.ctypes.data_as(C.c_void_p),
                                                  b.ctypes.data_as(C.c_void_p), cap, None, None))
        return a[: nw.value], b[: nn.value]

    def debug_tree(self):
        """(order int32 [n], keys uint64 [n], nodes_i int64 [nodes,4], nodes_d f64 [nodes,16])."""
        nn = C.c_int64(0)
        check(self.ctx, self.L.pbh_debug_tree(self.ctx, None, None, 0, None, None, C.byref(nn)))
        order = np.zeros(self.n, dtype=np.int32)
        keys = np.zeros(self.n, dtype=np.uint64)
        ni = np.zeros((nn.value, 4), dtype=np.int64)
        nd = np.zeros((nn.value, 16), dtype=np.float64)
        check(self.ctx, self.L.pbh_debug_tree(self.ctx, order.ctypes.data_as(C.c_void_p),
                                              keys.ctypes.data_as(C.c_void_p), nn.value,
                                              ni.ctypes.data_as(C.c_void_p),
                                              nd.ctypes.data_as(C.c_void_p), C.byref(nn)))
        return order, keys, ni, nd
