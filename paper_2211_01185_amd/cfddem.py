"""Thin ctypes binding of libcfddem (C ABI in include/cfddem.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of ``lib/libcfddem.so``.  PyTorch provides device memory (the
workspace and the input/output tensors) and the stream.  There is no CPU
fallback: importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libcfddem.so")
ABI_VERSION = 5

DEM_OK = 0
DEM_E_ARG = -1
DEM_E_WORKSPACE = -2
DEM_E_HIP = -3
DEM_E_DOMAIN = -4
DEM_E_CAPACITY = -5
DEM_E_NAN = -6
DEM_E_UNSUPPORTED = -7
DEM_E_ABI = -8

FP64 = 0
FP32_FORCES = 1

DRAG = {"difelice": 0, "dallavalle": 1, "rong": 2, "koch_hill": 3, "beetstra": 4, "gidaspow": 5}

SYMBOLS = ("dem_workspace_bytes", "dem_create", "dem_step", "cfd_dem_couple", "dem_read_state",
           "dem_read_forces", "dem_read_cells", "dem_read_contacts", "dem_poll", "dem_kinetic_energy",
           "dem_checkpoint_bytes", "dem_read_checkpoint", "dem_write_state", "dem_kinetic_energy_noalloc", "dem_metrics",

           "dem_kernel_timing",
           "dem_kernel_timing_read", "dem_destroy", "dem_batch_workspace_bytes", "dem_batch_create",
           "dem_batch_step", "dem_batch_couple", "dem_batch_run", "dem_batch_destroy",
           "dem_batch_slots_workspace_bytes", "dem_batch_create_slots", "dem_batch_admit", "dem_batch_retire",
           "dem_status_string")


class DemParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("precision", C.c_int32), ("n", C.c_int64),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("gravity", C.c_double * 3),
        ("dt", C.c_double),
        ("E", C.c_double), ("nu", C.c_double), ("e", C.c_double), ("mu", C.c_double),
        ("E_w", C.c_double), ("nu_w", C.c_double), ("e_w", C.c_double), ("mu_w", C.c_double),
        ("max_neighbors", C.c_int32), ("cell_capacity", C.c_int32), ("resort_every", C.c_int32),
        ("lanes", C.c_int32), ("d_max", C.c_double), ("d_min", C.c_double), ("skin", C.c_double),
        ("mu_r", C.c_double), ("mu_r_w", C.c_double),
    ]


class CfdParams(C.Structure):
    _fields_ = [
        ("order", C.c_int32), ("n_el", C.c_int32 * 3), ("rho_f", C.c_double), ("mu_f", C.c_double),
        ("drag", C.c_int32), ("model", C.c_int32), ("eps_min", C.c_double),
        ("shear", C.c_int32), ("smooth", C.c_int32), ("smooth_L2", C.c_double),
        ("elem_threads", C.c_int32),
    ]


class BatchLimits(C.Structure):
    _fields_ = [("slots", C.c_int32), ("couples", C.c_int32), ("max_particles", C.c_int64),
                ("max_elements", C.c_int64)]


class CfddemError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def load():
    """Load libcfddem.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2211_01185_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
    lib.dem_workspace_bytes.restype = C.c_size_t
    lib.dem_workspace_bytes.argtypes = [C.POINTER(DemParams), C.POINTER(CfdParams)]
    lib.dem_create.restype = i32
    lib.dem_create.argtypes = [C.POINTER(DemParams), C.POINTER(CfdParams), vp, vp, vp, vp, vp, vp,
                               C.c_size_t, vp, C.POINTER(vp)]
    lib.dem_step.restype = i32
    lib.dem_step.argtypes = [vp, i32, vp]
    lib.cfd_dem_couple.restype = i32
    lib.cfd_dem_couple.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dem_read_state.restype = i32
    lib.dem_read_state.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.dem_read_forces.restype = i32
    lib.dem_read_forces.argtypes = [vp, vp, vp, vp]
    lib.dem_read_cells.restype = i32
    lib.dem_read_cells.argtypes = [vp, vp, vp, C.POINTER(i32), vp]
    lib.dem_kinetic_energy.restype = i32
    lib.dem_kinetic_energy.argtypes = [vp, C.POINTER(dbl), vp]
    lib.dem_kinetic_energy_noalloc.restype = i32
    lib.dem_kinetic_energy_noalloc.argtypes = [vp, vp, vp]
    lib.dem_metrics.restype = i32
    lib.dem_metrics.argtypes = [vp, vp, vp, vp]
    lib.dem_read_contacts.restype = i32
    lib.dem_read_contacts.argtypes = [vp, vp, vp, i64, C.POINTER(i64), vp]
    lib.dem_poll.restype = i32
    lib.dem_poll.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), vp]
    lib.dem_checkpoint_bytes.restype = C.c_size_t
    lib.dem_checkpoint_bytes.argtypes = [vp]
    lib.dem_read_checkpoint.restype = i32
    lib.dem_read_checkpoint.argtypes = [vp, vp, C.c_size_t, vp]
    lib.dem_write_state.restype = i32
    lib.dem_write_state.argtypes = [vp, vp, C.c_size_t, vp]
    lib.dem_kernel_timing.restype = i32
    lib.dem_kernel_timing.argtypes = [vp, i32]
    lib.dem_kernel_timing_read.restype = i32
    lib.dem_kernel_timing_read.argtypes = [vp, C.POINTER(i64), C.POINTER(dbl), vp]
    lib.dem_destroy.restype = i32
    lib.dem_destroy.argtypes = [vp]
    lib.dem_batch_workspace_bytes.restype = C.c_size_t
    lib.dem_batch_workspace_bytes.argtypes = [i32, vp]
    lib.dem_batch_create.restype = i32
    lib.dem_batch_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.dem_batch_step.restype = i32
    lib.dem_batch_step.argtypes = [vp, i32, vp]
    lib.dem_batch_couple.restype = i32
    lib.dem_batch_couple.argtypes = [vp, vp]
    lib.dem_batch_run.restype = i32
    lib.dem_batch_run.argtypes = [vp, i32, i32, i32, vp]
    lib.dem_batch_destroy.restype = i32
    lib.dem_batch_destroy.argtypes = [vp]
    lib.dem_batch_slots_workspace_bytes.restype = C.c_size_t
    lib.dem_batch_slots_workspace_bytes.argtypes = [C.POINTER(BatchLimits)]
    lib.dem_batch_create_slots.restype = i32
    lib.dem_batch_create_slots.argtypes = [C.POINTER(BatchLimits), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.dem_batch_admit.restype = i32
    lib.dem_batch_admit.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dem_batch_retire.restype = i32
    lib.dem_batch_retire.argtypes = [vp, i32]
    lib.dem_status_string.restype = C.c_char_p
    lib.dem_status_string.argtypes = [i32]
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().dem_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != DEM_OK:
        raise CfddemError(status, where)


def make_params(dem: dict, fluid: dict, n: int, d_max: float, d_min: float, precision="fp64",
                max_neighbors=0, cell_capacity=0, resort_every=0, skin=0.0, lanes=0, elem_threads=0):
    """Fill the two C parameter structs from plain dicts (see synth.Workload)."""
    dp = DemParams()
    dp.abi_version = ABI_VERSION
    dp.precision = FP32_FORCES if precision in ("fp32", FP32_FORCES) else FP64
    dp.n = int(n)
    dp.box_lo[:] = [float(v) for v in dem["box_lo"]]
    dp.box_hi[:] = [float(v) for v in dem["box_hi"]]
    dp.gravity[:] = [float(v) for v in dem["gravity"]]
    dp.dt = float(dem["dt"])
    for k in ("E", "nu", "e", "mu"):
        setattr(dp, k, float(dem[k]))
        setattr(dp, k + "_w", float(dem.get(k + "_w", dem[k])))
    dp.max_neighbors = int(max_neighbors)
    dp.cell_capacity = int(cell_capacity)
    dp.resort_every = int(resort_every)
    dp.lanes = int(lanes)
    dp.d_max = float(d_max)
    dp.d_min = float(d_min)
    dp.skin = float(skin)
    dp.mu_r = float(dem.get("mu_r", 0.0))
    dp.mu_r_w = float(dem.get("mu_r_w", dem.get("mu_r", 0.0)))
    cp = CfdParams()
    cp.order = int(fluid["order"])
    cp.n_el[:] = [int(v) for v in fluid["n_el"]]
    cp.rho_f = float(fluid["rho_f"])
    cp.mu_f = float(fluid["mu_f"])
    drag = fluid.get("drag", 0)
    cp.drag = (DRAG[drag] if isinstance(drag, str) else int(drag)) | (0x100 if fluid.get("beta_over_eps") else 0)
    cp.model = int(fluid.get("model", 0))
    cp.eps_min = float(fluid.get("eps_min", 0.1))
    cp.shear = 1 if fluid.get("shear") else 0
    L2 = fluid.get("smooth_L2")
    cp.smooth = 0 if L2 is None else 1
    cp.smooth_L2 = 0.0 if L2 is None else float(L2)
    cp.elem_threads = int(elem_threads)
    return dp, cp


def workspace_bytes(dp: DemParams, cp: CfdParams) -> int:
    return int(load().dem_workspace_bytes(C.byref(dp), C.byref(cp)))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Bed:
    """One bed on the GPU: a dem_ctx plus the torch-owned workspace."""

    def __init__(self, dem: dict, fluid: dict, x, v, w, radius, density, precision="fp64",
                 max_neighbors=0, cell_capacity=0, resort_every=0, skin=0.0, lanes=0, elem_threads=0,
                 device="cuda", stream=None):
        import torch

        self._torch = torch
        lib = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        x = torch.as_tensor(np.asarray(x) if not torch.is_tensor(x) else x, **f64).contiguous()
        v = torch.as_tensor(np.asarray(v) if not torch.is_tensor(v) else v, **f64).contiguous()
        w = torch.as_tensor(np.asarray(w) if not torch.is_tensor(w) else w, **f64).contiguous()
        r = torch.as_tensor(np.asarray(radius) if not torch.is_tensor(radius) else radius, **f64).contiguous()
        rho = torch.as_tensor(np.asarray(density) if not torch.is_tensor(density) else density, **f64).contiguous()
        self.n = int(x.shape[1])
        if x.shape != (3, self.n) or v.shape != (3, self.n) or w.shape != (3, self.n):
            raise ValueError("x, v, w must be (3, n)")
        if r.shape != (self.n,) or rho.shape != (self.n,):
            raise ValueError("radius and density must be (n,)")
        rr = r.detach().cpu().numpy()
        self.dp, self.cp = make_params(dem, fluid, self.n, 2.0 * float(rr.max()), 2.0 * float(rr.min()),
                                       precision, max_neighbors, cell_capacity, resort_every, skin, lanes,
                                       elem_threads)
        nbytes = workspace_bytes(self.dp, self.cp)
        if nbytes == 0:
            raise CfddemError(DEM_E_ARG, "dem_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = C.c_void_p(self.workspace.data_ptr() + off)
        self._ws_len = nbytes
        n_el = [int(v) for v in fluid["n_el"]]
        self.n_elem = n_el[0] * n_el[1] * n_el[2]
        self.nq = (int(fluid["order"]) + 1) ** 3
        self._h = C.c_void_p()
        st = C.c_void_p(self.stream.cuda_stream)
        _check(lib.dem_create(C.byref(self.dp), C.byref(self.cp), _ptr(x), _ptr(v), _ptr(w), _ptr(r),
                              _ptr(rho), self._ws_ptr, C.c_size_t(nbytes), st, C.byref(self._h)),
               "dem_create")
        self.stream.synchronize()
        self._lib = lib

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            self._lib.dem_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _st(self):
        return C.c_void_p(self.stream.cuda_stream)

    # -- hot path ---------------------------------------------------------
    def step(self, n_steps: int = 1):
        _check(self._lib.dem_step(self._h, int(n_steps), self._st), "dem_step")

    def couple(self, U, P, out=None, elem_sums=False):
        """One coupling step.  U: (3, n_v) and P: (n_p,) float64 device tensors.
        Returns a dict of device tensors (eps_q, beta_q, fpf_q[, elem_sums])."""
        torch = self._torch
        if out is None:
            m = self.n_elem * self.nq
            out = dict(eps_q=torch.empty(m, dtype=torch.float64, device=self.device),
                       beta_q=torch.empty(m, dtype=torch.float64, device=self.device),
                       fpf_q=torch.empty((3, m), dtype=torch.float64, device=self.device))
            if elem_sums:
                out["elem_sums"] = torch.empty((12, self.n_elem), dtype=torch.float64, device=self.device)
        _check(self._lib.cfd_dem_couple(self._h, _ptr(U), _ptr(P), _ptr(out["eps_q"]), _ptr(out["beta_q"]),
                                        _ptr(out["fpf_q"]), _ptr(out.get("elem_sums")), self._st),
               "cfd_dem_couple")
        return out

    # -- accessors (original-ID order) -------------------------------------
    def read_state(self):
        torch = self._torch
        out = {k: torch.empty((3, self.n), dtype=torch.float64, device=self.device) for k in ("x", "v", "w", "ffp")}
        _check(self._lib.dem_read_state(self._h, _ptr(out["x"]), _ptr(out["v"]), _ptr(out["w"]), _ptr(out["ffp"]),
                                        self._st), "dem_read_state")
        return out

    def read_forces(self):
        torch = self._torch
        F = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        T = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        _check(self._lib.dem_read_forces(self._h, _ptr(F), _ptr(T), self._st), "dem_read_forces")
        return F, T

    def kinetic_energy(self):
        """(translational, rotational) kinetic energy of the current state;
        synchronizes the bed's stream."""
        out = (C.c_double * 2)()
        _check(self._lib.dem_kinetic_energy(self._h, out, self._st), "dem_kinetic_energy")
        return float(out[0]), float(out[1])

    def metrics(self, eps_q=None):
        """Monitoring metrics of the current state (dem_metrics): total
        momentum, largest overlap over the smaller radius, solid volume of the
        particles and, given the eps_q of a coupling step, the solid volume at
        the quadrature points; synchronizes the bed's stream."""
        out = (C.c_double * 7)()
        _check(self._lib.dem_metrics(self._h, _ptr(eps_q), out, self._st), "dem_metrics")
        return {"momentum": (float(out[0]), float(out[1]), float(out[2])), "max_overlap_over_radius": float(out[3]),
                "solid_volume": float(out[4]), "solid_volume_at_quadrature_points": float(out[5]),
                "max_speed": float(out[6])}

    def read_cells(self):
        torch = self._torch
        elem = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cell = torch.empty(self.n, dtype=torch.int32, device=self.device)
        k = (C.c_int32 * 3)()
        _check(self._lib.dem_read_cells(self._h, _ptr(elem), _ptr(cell), k, self._st), "dem_read_cells")
        return elem, cell, [k[0], k[1], k[2]]

    def read_contacts(self):
        """(i, j, delta_t) as numpy arrays sorted by (i, j); j = -1-w for walls."""
        torch = self._torch
        total = C.c_int64()
        _check(self._lib.dem_read_contacts(self._h, None, None, 0, C.byref(total), self._st),
               "dem_read_contacts")
        cap = max(int(total.value), 1)
        pairs = torch.empty((2, cap), dtype=torch.int64, device=self.device)
        dt = torch.empty((3, cap), dtype=torch.float64, device=self.device)
        _check(self._lib.dem_read_contacts(self._h, _ptr(pairs), _ptr(dt), cap, C.byref(total), self._st),
               "dem_read_contacts")
        m = int(total.value)
        pairs = pairs[:, :m].cpu().numpy()
        dt = dt[:, :m].cpu().numpy()
        return pairs[0], pairs[1], dt.T.copy()

    def checkpoint(self):
        """The bed's full state as a uint8 device tensor (dem_read_checkpoint)."""
        torch = self._torch
        nbytes = int(self._lib.dem_checkpoint_bytes(self._h))
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        blob = buf[off:off + nbytes]
        _check(self._lib.dem_read_checkpoint(self._h, C.c_void_p(blob.data_ptr()), C.c_size_t(nbytes), self._st),
               "dem_read_checkpoint")
        return blob

    def restore(self, blob):
        """Replace the bed's state by a checkpoint (a uint8 tensor on any
        device, as returned by checkpoint(); copied to a 256-byte aligned
        device buffer first when needed)."""
        torch = self._torch
        nbytes = int(blob.numel())
        if blob.device != self.device or blob.data_ptr() % 256:
            buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            buf[off:off + nbytes].copy_(blob)
            blob = buf[off:off + nbytes]
        _check(self._lib.dem_write_state(self._h, C.c_void_p(blob.data_ptr()), C.c_size_t(nbytes), self._st),
               "dem_write_state")

    def poll(self):
        """(sticky_error, n_contacts); synchronizes the stream."""
        err = C.c_int32()
        nc = C.c_int64()
        self._lib.dem_poll(self._h, C.byref(err), C.byref(nc), self._st)
        return int(err.value), int(nc.value)

    def kernel_timing(self, enable: bool):
        _check(self._lib.dem_kernel_timing(self._h, 1 if enable else 0), "dem_kernel_timing")

    def kernel_timing_read(self):
        """(launches, total_ms) of the contact-force kernel since the last read."""
        launches = C.c_int64()
        ms = C.c_double()
        _check(self._lib.dem_kernel_timing_read(self._h, C.byref(launches), C.byref(ms), self._st),
               "dem_kernel_timing_read")
        return int(launches.value), float(ms.value)


class Batch:
    """Beds advanced together by shared launches (dem_batch_*).

    fields: None (no coupling) or one (U, P) pair of float64 device tensors per
    bed; the coupling outputs are allocated here, one dict per bed, and
    rewritten by every couple() / run(couple=True)."""

    def __init__(self, beds, fields=None, elem_sums=False, stream=None):
        import torch

        self._torch = torch
        lib = load()
        self.beds = list(beds)
        nb = len(self.beds)
        self.stream = stream if stream is not None else self.beds[0].stream
        self.device = self.beds[0].device
        handles = (C.c_void_p * nb)(*[b._h.value for b in self.beds])
        nbytes = int(lib.dem_batch_workspace_bytes(nb, handles))
        if nbytes == 0:
            raise CfddemError(DEM_E_ARG, "dem_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        ws = C.c_void_p(self.workspace.data_ptr() + off)
        self.out = None
        arrays = [None] * 6
        if fields is not None:
            if len(fields) != nb:
                raise ValueError("one (U, P) pair per bed")
            self.fields = [(U.contiguous(), P.contiguous()) for U, P in fields]
            self.out = []
            for bed in self.beds:
                m = bed.n_elem * bed.nq
                o = dict(eps_q=torch.empty(m, dtype=torch.float64, device=self.device),
                         beta_q=torch.empty(m, dtype=torch.float64, device=self.device),
                         fpf_q=torch.empty((3, m), dtype=torch.float64, device=self.device))
                if elem_sums:
                    o["elem_sums"] = torch.empty((12, bed.n_elem), dtype=torch.float64, device=self.device)
                self.out.append(o)

            def ptrs(ts):
                return (C.c_void_p * nb)(*[t.data_ptr() if t is not None else None for t in ts])

            arrays = [ptrs([f[0] for f in self.fields]), ptrs([f[1] for f in self.fields]),
                      ptrs([o["eps_q"] for o in self.out]), ptrs([o["beta_q"] for o in self.out]),
                      ptrs([o["fpf_q"] for o in self.out]),
                      ptrs([o.get("elem_sums") for o in self.out]) if elem_sums else None]
        self._h = C.c_void_p()
        _check(lib.dem_batch_create(nb, handles, *arrays, ws, C.c_size_t(nbytes), self._st, C.byref(self._h)),
               "dem_batch_create")
        self._lib = lib

    @property
    def _st(self):
        return C.c_void_p(self.stream.cuda_stream)

    def step(self, n_steps: int = 1):
        _check(self._lib.dem_batch_step(self._h, int(n_steps), self._st), "dem_batch_step")

    def couple(self):
        _check(self._lib.dem_batch_couple(self._h, self._st), "dem_batch_couple")
        return self.out

    def run(self, n_chunks: int, steps_per_chunk: int, couple: bool = True):
        """n_chunks x [couple] + steps_per_chunk steps, replayed from one HIP graph."""
        _check(self._lib.dem_batch_run(self._h, int(n_chunks), int(steps_per_chunk), 1 if couple else 0,
                                       self._st), "dem_batch_run")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            self._lib.dem_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlotBatch:
    """A batch with fixed slots that beds join and leave while it runs
    (dem_batch_create_slots / dem_batch_admit / dem_batch_retire): the
    continuous-batching form used by the server.  admit() returns the bed's
    coupling outputs (a dict of device tensors rewritten by every coupling
    step of the batch)."""

    def __init__(self, slots, max_particles, max_elements=0, couples=True, device="cuda", stream=None):
        import torch

        self._torch = torch
        lib = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.limits = BatchLimits(int(slots), 1 if couples else 0, int(max_particles), int(max_elements))
        nbytes = int(lib.dem_batch_slots_workspace_bytes(C.byref(self.limits)))
        if nbytes == 0:
            raise CfddemError(DEM_E_ARG, "dem_batch_slots_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._h = C.c_void_p()
        self._lib = lib
        _check(lib.dem_batch_create_slots(C.byref(self.limits), C.c_void_p(self.workspace.data_ptr() + off),
                                          C.c_size_t(nbytes), self._st, C.byref(self._h)), "dem_batch_create_slots")
        self.held = {}  # slot -> (bed, fields, outputs)

    @property
    def _st(self):
        return C.c_void_p(self.stream.cuda_stream)

    def admit(self, slot, bed, fields=None, elem_sums=False):
        torch = self._torch
        out = None
        args = [None] * 6
        if self.limits.couples:
            U, P = (t.contiguous() for t in fields)
            m = bed.n_elem * bed.nq
            out = dict(eps_q=torch.empty(m, dtype=torch.float64, device=self.device),
                       beta_q=torch.empty(m, dtype=torch.float64, device=self.device),
                       fpf_q=torch.empty((3, m), dtype=torch.float64, device=self.device))
            if elem_sums:
                out["elem_sums"] = torch.empty((12, bed.n_elem), dtype=torch.float64, device=self.device)
            fields = (U, P)
            args = [_ptr(U), _ptr(P), _ptr(out["eps_q"]), _ptr(out["beta_q"]), _ptr(out["fpf_q"]),
                    _ptr(out.get("elem_sums"))]
        _check(self._lib.dem_batch_admit(self._h, int(slot), bed._h, *args, self._st), "dem_batch_admit")
        self.held[int(slot)] = (bed, fields, out)
        return out

    def retire(self, slot):
        _check(self._lib.dem_batch_retire(self._h, int(slot)), "dem_batch_retire")
        return self.held.pop(int(slot))

    def step(self, n_steps: int = 1):
        _check(self._lib.dem_batch_step(self._h, int(n_steps), self._st), "dem_batch_step")

    def couple(self):
        _check(self._lib.dem_batch_couple(self._h, self._st), "dem_batch_couple")

    def run(self, n_chunks: int, steps_per_chunk: int, couple: bool = True):
        _check(self._lib.dem_batch_run(self._h, int(n_chunks), int(steps_per_chunk), 1 if couple else 0,
                                       self._st), "dem_batch_run")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            self._lib.dem_batch_destroy(self._h)
            self._h = C.c_void_p()
            self.held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bed_from_workload(wl, precision=None, device="cuda", **kw) -> Bed:
    """Create a Bed from a synth.Workload (positions etc. copied to the GPU)."""
    prec = precision if precision is not None else wl.run.get("precision", "fp64")
    return Bed(wl.dem, wl.fluid, wl.x, wl.v, wl.w, wl.radius, wl.density, precision=prec, device=device, **kw)
