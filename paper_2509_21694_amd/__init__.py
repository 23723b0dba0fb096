"""Python binding of libmpip (ctypes; argument marshalling only).

Every step of an evaluation runs in the library's HIP kernels on the GPU;
PyTorch provides device memory and the current HIP stream.  If the built
library is missing this module raises at import time -- there is no CPU
fallback.

Method: arxiv 2509.21694 -- depth pruning (evaluate the first K of T layers,
Methods "Message Passing Depth Pruning") and halo partitions (root atoms
first, Methods "Graph Partitioning" / "Global Output Integration").
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpip.so")

FP32 = 0
BF16_MIXED = 1
PRECISIONS = {"fp32": FP32, "bf16": BF16_MIXED, FP32: FP32, BF16_MIXED: BF16_MIXED}

OK, EINVAL, ECELL, ECAPACITY, EDEVICE, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ECELL", -3: "ECAPACITY", -4: "EDEVICE",
                -5: "ENOMEM", -6: "EUNSUPPORTED"}


class MpipError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class HParamsC(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("l_max", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("n_basis", ctypes.c_int32), ("envelope_p", ctypes.c_int32),
                ("radial_hidden", ctypes.c_int32), ("r_cut", ctypes.c_double),
                ("inv_avg_neighbors", ctypes.c_double)]


class SystemC(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("n_owned", ctypes.c_int64), ("positions", ctypes.c_void_p),
                ("species", ctypes.c_void_p), ("cell", ctypes.c_double * 9), ("pbc", ctypes.c_uint8 * 3)]


class OutputsC(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_void_p), ("forces", ctypes.c_void_p), ("virial", ctypes.c_void_p),
                ("atom_energy", ctypes.c_void_p)]


MAX_PHASES = 48


class TimingC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("name", (ctypes.c_char * 24) * MAX_PHASES),
                ("ms", ctypes.c_double * MAX_PHASES), ("calls", ctypes.c_int64 * MAX_PHASES)]


class MdParamsC(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("n_steps", ctypes.c_int64), ("friction", ctypes.c_double),
                ("temperature", ctypes.c_double), ("seed", ctypes.c_uint64), ("skin", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2509_21694_amd/build.py`")
    # PyTorch ships its own HIP runtime under the same soname: loading it
    # first makes the library bind to that runtime, so the process holds one
    # HIP runtime whose streams and memory both sides share
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ, V = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    lib.mpip_weights_count.argtypes = [P(HParamsC)]
    lib.mpip_weights_count.restype = SZ
    lib.mpip_model_create.argtypes = [P(HParamsC), P(ctypes.c_float), SZ, I32, P(V)]
    lib.mpip_model_create.restype = I32
    lib.mpip_model_destroy.argtypes = [V]
    lib.mpip_model_destroy.restype = I32
    lib.mpip_workspace_size.argtypes = [V, P(SystemC), I32, I32, I64, P(SZ)]
    lib.mpip_workspace_size.restype = I32
    lib.mpip_evaluate.argtypes = [V, P(SystemC), I32, I32, V, V, SZ, I64, P(OutputsC)]
    lib.mpip_evaluate.restype = I32
    lib.mpip_evaluate_noalloc.argtypes = [V, P(SystemC), I32, I32, V, I64, P(OutputsC)]
    lib.mpip_evaluate_noalloc.restype = I32
    lib.mpip_workspace_status.argtypes = [V, V, P(I64)]
    lib.mpip_workspace_status.restype = I32
    lib.mpip_neighbor_workspace_size.argtypes = [I64, I64]
    lib.mpip_neighbor_workspace_size.restype = SZ
    lib.mpip_neighbor_list.argtypes = [P(SystemC), ctypes.c_double, V, V, SZ, I64, V, V, V, P(I64)]
    lib.mpip_neighbor_list.restype = I32
    lib.mpip_coupling_tensor.argtypes = [I32, I32, I32, P(ctypes.c_double)]
    lib.mpip_coupling_tensor.restype = I32
    lib.mpip_radial_table.argtypes = [P(HParamsC), P(ctypes.c_float), SZ, I32, P(ctypes.c_uint32)]
    lib.mpip_radial_table.restype = I32
    lib.mpip_timing_enable.argtypes = [V, I32]
    lib.mpip_timing_enable.restype = I32
    lib.mpip_timing_read.argtypes = [V, P(TimingC)]
    lib.mpip_timing_read.restype = I32
    lib.mpip_slab_workspace_size.argtypes = [I64, ctypes.c_double, ctypes.c_double]
    lib.mpip_slab_workspace_size.restype = SZ
    lib.mpip_slab_share.argtypes = [V, V, I64, P(ctypes.c_double), I32, I32, I32, ctypes.c_double, V, V, SZ, I64,
                                    V, V, V, P(I64), P(I64)]
    lib.mpip_slab_share.restype = I32
    lib.mpip_accumulate_rows.argtypes = [V, V, I64, I64, V, V]
    lib.mpip_accumulate_rows.restype = I32
    lib.mpip_batch_workspace_size.argtypes = [V, I64, I32, I32, I32, I64, P(SZ)]
    lib.mpip_batch_workspace_size.restype = I32
    lib.mpip_evaluate_batch.argtypes = [V, I32, P(I64), V, V, P(ctypes.c_double), P(ctypes.c_uint8), I32, I32, V, V,
                                        SZ, I64, V, V, V]
    lib.mpip_evaluate_batch.restype = I32
    lib.mpip_md_workspace_size.argtypes = [V, P(SystemC), P(MdParamsC), I32, I32, I64, P(SZ)]
    lib.mpip_md_workspace_size.restype = I32
    lib.mpip_md_run.argtypes = [V, P(SystemC), V, V, V, V, P(MdParamsC), I32, I32, V, V, SZ, I64, V, V]
    lib.mpip_md_run.restype = I32
    lib.mpip_partitioned_workspace_size.argtypes = [V, P(SystemC), I32, I32, I32, I32, ctypes.c_double, I64, I64,
                                                    I64, P(SZ)]
    lib.mpip_partitioned_workspace_size.restype = I32
    lib.mpip_evaluate_partitioned.argtypes = [V, P(SystemC), I32, I32, I32, I32, ctypes.c_double, I64, V, V, SZ,
                                              I64, I64, P(OutputsC), P(I64)]
    lib.mpip_evaluate_partitioned.restype = I32
    lib.mpip_bfs_share_workspace_size.argtypes = [I64, ctypes.c_double, I32, ctypes.c_double, I64]
    lib.mpip_bfs_share_workspace_size.restype = SZ
    lib.mpip_bfs_share.argtypes = [P(SystemC), ctypes.c_double, I32, I32, I32, I32, V, V, SZ, I64, I64, V, V, V,
                                   P(I64), P(I64), P(I64)]
    lib.mpip_bfs_share.restype = I32
    lib.mpip_last_error.argtypes = []
    lib.mpip_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTED = ["mpip_weights_count", "mpip_model_create", "mpip_model_destroy", "mpip_workspace_size",
            "mpip_evaluate", "mpip_workspace_status", "mpip_neighbor_workspace_size",
            "mpip_neighbor_list", "mpip_coupling_tensor", "mpip_radial_table", "mpip_timing_enable",
            "mpip_timing_read",
            "mpip_slab_workspace_size", "mpip_slab_share", "mpip_accumulate_rows",
            "mpip_batch_workspace_size", "mpip_evaluate_batch", "mpip_md_workspace_size", "mpip_md_run",
            "mpip_partitioned_workspace_size", "mpip_evaluate_partitioned", "mpip_bfs_share_workspace_size",
            "mpip_bfs_share", "mpip_evaluate_noalloc", "mpip_last_error"]

# size of the library's static workspace used by mpip_evaluate_noalloc (MPIP_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 256 << 20


def _check(st: int):
    if st != OK:
        raise MpipError(st, lib.mpip_last_error().decode())


def hparams_c(hp) -> HParamsC:
    return HParamsC(hp.n_species, hp.n_layers, hp.l_max, hp.channels, hp.n_basis, hp.envelope_p,
                    hp.radial_hidden, float(hp.r_cut), float(1.0 / hp.avg_neighbors))


def weights_count(hp) -> int:
    return int(lib.mpip_weights_count(ctypes.byref(hparams_c(hp))))


def coupling_tensor(l1: int, l2: int, l3: int) -> np.ndarray:
    out = np.zeros((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1), dtype=np.float64)
    _check(lib.mpip_coupling_tensor(l1, l2, l3, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1)


# intervals of the radial table over [0, r_cut]
RADIAL_TABLE_INTERVALS = 4096


def radial_table(hp, weights: np.ndarray, layer: int) -> np.ndarray:
    """The BF16 form's radial table of one layer: uint32 [4096, radial_hidden]
    (low half BF16 a(d_k), high half BF16 a(d_k+1) - a(d_k))."""
    w = np.ascontiguousarray(weights, dtype=np.float32)
    out = np.zeros((RADIAL_TABLE_INTERVALS, hp.radial_hidden), dtype=np.uint32)
    _check(lib.mpip_radial_table(ctypes.byref(hparams_c(hp)), w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                 w.size, int(layer), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return out


def _system(positions, species, cell, pbc, n_owned) -> SystemC:
    s = SystemC()
    s.n_atoms = int(positions.shape[0])
    s.n_owned = int(positions.shape[0] if n_owned is None else n_owned)
    s.positions = positions.data_ptr()
    s.species = species.data_ptr()
    c = np.asarray(cell, dtype=np.float64).reshape(9)
    for k in range(9):
        s.cell[k] = float(c[k])
    for k in range(3):
        s.pbc[k] = 1 if bool(np.asarray(pbc)[k]) else 0
    return s


def _stream_ptr(torch, device, stream=None) -> int:
    st = torch.cuda.current_stream(device) if stream is None else stream
    return int(st.cuda_stream)


def estimate_edges(n_atoms: int, cell, r_cut: float) -> int:
    """Edge capacity guess from the mean density of the cell (x1.6 + margin)."""
    vol = abs(float(np.linalg.det(np.asarray(cell, dtype=np.float64))))
    dens = n_atoms / vol if vol > 0 else 0.1
    deg = dens * 4.0 / 3.0 * math.pi * r_cut ** 3
    return int(n_atoms * max(48.0, 1.6 * deg)) + 1024


class Model:
    """A weight set on one GPU.  ``hp`` has the fields of workloads.HParams."""

    def __init__(self, hp, weights: np.ndarray, device: int = 0):
        import torch
        self.torch = torch
        self.hp = hp
        self.device = torch.device("cuda", device)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        self._hpc = hparams_c(hp)
        h = ctypes.c_void_p()
        _check(lib.mpip_model_create(ctypes.byref(self._hpc), w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     w.size, device, ctypes.byref(h)))
        self._h = h
        self._ws = None
        self._ws_key = None

    def __del__(self, _destroy=lib.mpip_model_destroy):
        # the library function is bound at class creation: at interpreter
        # shutdown the module global ``lib`` may already be None
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            self._h = None

    def workspace_bytes(self, n_atoms: int, K: int, precision, max_edges: int) -> int:
        s = SystemC()
        s.n_atoms = n_atoms
        s.n_owned = n_atoms
        out = ctypes.c_size_t()
        _check(lib.mpip_workspace_size(self._h, ctypes.byref(s), PRECISIONS[precision], K, max_edges,
                                       ctypes.byref(out)))
        return int(out.value)

    def workspace(self, n_atoms: int, K: int, precision, max_edges: int):
        nbytes = self.workspace_bytes(n_atoms, K, precision, max_edges)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        return self._ws

    def evaluate(self, positions, species, cell, pbc=(True, True, True), K: Optional[int] = None,
                 precision="fp32", n_owned: Optional[int] = None, atom_energy: bool = False,
                 max_edges: Optional[int] = None, out=None, stream=None, check: bool = True):
        """Energy / forces / virial of one system.  ``positions``: cuda
        float64 [N,3]; ``species``: cuda int32 [N].  Returns a dict of cuda
        tensors (energy [1], forces [N,3], virial [3,3], atom_energy [N])
        plus ``n_edges`` when ``check`` is set (synchronises the stream)."""
        torch = self.torch
        K = self.hp.n_layers if K is None else int(K)
        N = int(positions.shape[0])
        assert positions.dtype == torch.float64 and positions.is_cuda and positions.is_contiguous()
        assert species.dtype == torch.int32 and species.is_cuda and species.is_contiguous()
        if max_edges is None:
            max_edges = estimate_edges(N, cell, self.hp.r_cut)
        prec = PRECISIONS[precision]
        for attempt in range(2):
            ws = self.workspace(N, K, prec, max_edges)
            if out is None:
                o = {"energy": torch.empty(1, dtype=torch.float64, device=self.device),
                     "forces": torch.empty((N, 3), dtype=torch.float64, device=self.device),
                     "virial": torch.empty((3, 3), dtype=torch.float64, device=self.device),
                     "atom_energy": (torch.empty(N, dtype=torch.float64, device=self.device)
                                     if atom_energy else None)}
            else:
                o = out
            oc = OutputsC(o["energy"].data_ptr(), o["forces"].data_ptr(), o["virial"].data_ptr(),
                          o["atom_energy"].data_ptr() if o.get("atom_energy") is not None else None)
            sysc = _system(positions, species, cell, pbc, n_owned)
            sp = _stream_ptr(torch, self.device, stream)
            _check(lib.mpip_evaluate(self._h, ctypes.byref(sysc), prec, K, ctypes.c_void_p(sp),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), max_edges, ctypes.byref(oc)))
            if not check:
                if stream is not None:
                    # keep the caching allocator from handing the workspace or the
                    # outputs to other work while this stream may still use them
                    ws.record_stream(stream)
                    for v in o.values():
                        if isinstance(v, torch.Tensor):
                            v.record_stream(stream)
                return o
            ne = ctypes.c_int64()
            st = lib.mpip_workspace_status(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(sp), ctypes.byref(ne))
            if st == ECAPACITY and attempt == 0:
                max_edges = int(ne.value * 1.05) + 1024
                continue
            _check(st)
            o["n_edges"] = int(ne.value)
            return o
        raise MpipError(ECAPACITY, "edge capacity")


    def evaluate_noalloc(self, positions, species, cell, pbc, out, K: Optional[int] = None, precision="fp32",
                         n_owned: Optional[int] = None, max_edges: Optional[int] = None, stream=None):
        """mpip_evaluate_noalloc: the evaluation of ``evaluate`` with the
        library's static workspace; ``out`` is a dict of preallocated cuda
        tensors (energy [1], forces [N,3], virial [3,3], optional
        atom_energy [N]).  Nothing is allocated and nothing synchronised
        (except for partition shares, as in ``evaluate``); a data-dependent
        error leaves NaN in the energy and virial."""
        torch = self.torch
        K = self.hp.n_layers if K is None else int(K)
        N = int(positions.shape[0])
        assert positions.dtype == torch.float64 and positions.is_cuda and positions.is_contiguous()
        assert species.dtype == torch.int32 and species.is_cuda and species.is_contiguous()
        if max_edges is None:
            max_edges = estimate_edges(N, cell, self.hp.r_cut)
        oc = OutputsC(out["energy"].data_ptr(), out["forces"].data_ptr(), out["virial"].data_ptr(),
                      out["atom_energy"].data_ptr() if out.get("atom_energy") is not None else None)
        sysc = _system(positions, species, cell, pbc, n_owned)
        sp = _stream_ptr(torch, self.device, stream)
        _check(lib.mpip_evaluate_noalloc(self._h, ctypes.byref(sysc), PRECISIONS[precision], K,
                                         ctypes.c_void_p(sp), max_edges, ctypes.byref(oc)))
        return out

    def md_run(self, positions, velocities, species, masses, cell, pbc=(True, True, True), *, dt: float,
               n_steps: int, forces=None, friction: float = 0.0, temperature: float = 0.0, seed: int = 0,
               skin: float = 0.0, K: Optional[int] = None, precision="fp32", max_edges: Optional[int] = None,
               stream=None):
        """``n_steps`` MD steps on the device (mpip_md_run): BAOAB Langevin,
        velocity Verlet when ``friction`` is 0.  ``positions``, ``velocities``
        (cuda float64 [N,3]) are updated in place; ``skin`` > 0 reuses a
        neighbour list of radius r_cut + skin while no atom has moved more
        than skin/2 (same edges as a rebuild); ``forces`` (cuda float64
        [N,3]) must hold the forces at ``positions`` or be None (then they are
        evaluated first).  ``masses``: cuda float64 [n_species] (amu).
        Returns cuda tensors epot [n_steps], ekin [n_steps] (eV) and the
        final forces; synchronises the stream and raises on a data error."""
        torch = self.torch
        K = self.hp.n_layers if K is None else int(K)
        N = int(positions.shape[0])
        for t in (positions, velocities):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and tuple(t.shape) == (N, 3)
        assert masses.dtype == torch.float64 and masses.is_cuda and masses.numel() >= self.hp.n_species
        if max_edges is None:
            max_edges = int(estimate_edges(N, cell, self.hp.r_cut) * 1.1)
        if forces is None:
            first = self.evaluate(positions, species, cell, pbc, K=K, precision=precision, max_edges=max_edges,
                                  stream=stream)
            forces = first["forces"]
            # the list of the starting positions sets a floor under the capacity
            # (evaluate may have grown it on its retry)
            max_edges = max(max_edges, int(first["n_edges"] * 1.1) + 1024)
        prec = PRECISIONS[precision]
        sysc = _system(positions, species, cell, pbc, None)
        prm = MdParamsC(float(dt), int(n_steps), float(friction), float(temperature), int(seed), float(skin))
        need = ctypes.c_size_t()
        _check(lib.mpip_md_workspace_size(self._h, ctypes.byref(sysc), ctypes.byref(prm), prec, K, max_edges,
                                          ctypes.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = None
            self._ws = torch.empty(int(need.value), dtype=torch.uint8, device=self.device)
        ws = self._ws
        epot = torch.empty(max(n_steps, 1), dtype=torch.float64, device=self.device)
        ekin = torch.empty(max(n_steps, 1), dtype=torch.float64, device=self.device)
        sp = _stream_ptr(torch, self.device, stream)
        _check(lib.mpip_md_run(self._h, ctypes.byref(sysc), ctypes.c_void_p(positions.data_ptr()),
                               ctypes.c_void_p(velocities.data_ptr()), ctypes.c_void_p(forces.data_ptr()),
                               ctypes.c_void_p(masses.data_ptr()), ctypes.byref(prm), prec, K, ctypes.c_void_p(sp),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), max_edges,
                               ctypes.c_void_p(epot.data_ptr()), ctypes.c_void_p(ekin.data_ptr())))
        ne = ctypes.c_int64()
        _check(lib.mpip_workspace_status(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(sp), ctypes.byref(ne)))
        return epot[:n_steps], ekin[:n_steps], forces

    def evaluate_partitioned(self, positions, species, cell, pbc=(True, True, True), *, n_parts: int,
                             axis: int = 0, halo: Optional[float] = None, graph_halo: bool = False,
                             K: Optional[int] = None, precision="fp32", atom_energy: bool = False,
                             max_local: Optional[int] = None, max_edges: Optional[int] = None, stream=None):
        """Whole structure in ``n_parts`` slab partitions along ``axis``,
        evaluated one after the other on this GPU with one reused workspace
        (mpip_evaluate_partitioned); the halo is geometric with depth
        ``halo`` (default K r_cut), or the K-hop graph halo when
        ``graph_halo`` is set.  Returns a
        dict of cuda tensors (energy [1], forces [N,3], virial [3,3],
        atom_energy [N]) and ``parts``: numpy int64 [n_parts, 3] of (rows,
        roots, directed edges) per share.  Retries once with larger share
        capacities when a share outgrows the estimates."""
        torch = self.torch
        K = self.hp.n_layers if K is None else int(K)
        N = int(positions.shape[0])
        assert positions.dtype == torch.float64 and positions.is_cuda and positions.is_contiguous()
        assert species.dtype == torch.int32 and species.is_cuda and species.is_contiguous()
        if halo is None:
            halo = K * self.hp.r_cut
        c = np.asarray(cell, dtype=np.float64).reshape(3, 3)
        Lax = float(c[axis, axis])
        if max_local is None:
            max_local = min(int(N * (1.0 / n_parts + 2.0 * halo / Lax) * 1.05) + 1024,
                            N * (2 * (int(math.ceil(halo / Lax)) + 1) + 1))
        edges_given = max_edges is not None
        if not edges_given:
            max_edges = estimate_edges(N, cell, self.hp.r_cut) * max_local // N + 1024
        prec = PRECISIONS[precision]
        o = {"energy": torch.empty(1, dtype=torch.float64, device=self.device),
             "forces": torch.empty((N, 3), dtype=torch.float64, device=self.device),
             "virial": torch.empty((3, 3), dtype=torch.float64, device=self.device),
             "atom_energy": torch.empty(N, dtype=torch.float64, device=self.device) if atom_energy else None}
        oc = OutputsC(o["energy"].data_ptr(), o["forces"].data_ptr(), o["virial"].data_ptr(),
                      o["atom_energy"].data_ptr() if atom_energy else None)
        sysc = _system(positions, species, cell, pbc, None)
        sp = _stream_ptr(torch, self.device, stream)
        parts = np.zeros((n_parts, 3), dtype=np.int64)
        graph_edges = estimate_edges(N, cell, self.hp.r_cut) if graph_halo else -1
        # the driver stops at the first share that outgrows the capacities and
        # reports that share's sizes (later shares read zero), so a later,
        # larger share can overflow again: up to four retries, each growing
        # the capacities to at least what the last overflow needed
        attempts = 5
        for attempt in range(attempts):
            need = ctypes.c_size_t()
            _check(lib.mpip_partitioned_workspace_size(self._h, ctypes.byref(sysc), prec, K, n_parts, axis,
                                                       float(halo), graph_edges, max_local, max_edges,
                                                       ctypes.byref(need)))
            if self._ws is None or self._ws.numel() < need.value:
                self._ws = None
                self._ws = torch.empty(int(need.value), dtype=torch.uint8, device=self.device)
            st = lib.mpip_evaluate_partitioned(self._h, ctypes.byref(sysc), prec, K, n_parts, axis, float(halo),
                                               graph_edges, ctypes.c_void_p(sp), ctypes.c_void_p(self._ws.data_ptr()),
                                               self._ws.numel(), max_local, max_edges, ctypes.byref(oc),
                                               parts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            if st == ECAPACITY and attempt + 1 < attempts:
                if graph_halo and parts[:, 0].sum() == 0:     # the whole structure's list overflowed
                    graph_edges = max(graph_edges, int(parts[0, 2] * 1.05) + 1024)
                    continue
                max_local = max(max_local, int(parts[:, 0].max() * 1.05) + 1024)
                max_edges = max(max_edges, int(parts[:, 2].max() * 1.05) + 1024)
                if not edges_given:   # the default edge capacity follows the row capacity
                    max_edges = max(max_edges, estimate_edges(N, cell, self.hp.r_cut) * max_local // N + 1024)
                continue
            _check(st)
            o["parts"] = parts
            return o
        raise MpipError(ECAPACITY, "share capacity")


class Batch:
    """Device inputs of a batch of independent structures (atoms concatenated)."""

    def __init__(self, structures, device):
        import torch
        self.B = len(structures)
        counts = [int(np.asarray(s.positions).shape[0]) for s in structures]
        self.atom_ptr = np.ascontiguousarray(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))
        self.n_atoms = int(self.atom_ptr[-1])
        self.cells = np.ascontiguousarray(np.stack([np.asarray(s.cell, dtype=np.float64).reshape(9)
                                                    for s in structures]))
        self.pbc = np.ascontiguousarray(np.stack([np.asarray(s.pbc).astype(np.uint8).reshape(3)
                                                  for s in structures]))
        self.positions = torch.tensor(np.concatenate([s.positions for s in structures]), dtype=torch.float64,
                                      device=device)
        self.species = torch.tensor(np.concatenate([s.species for s in structures]).astype(np.int32),
                                    dtype=torch.int32, device=device)
        vol = np.abs(np.prod(self.cells[:, [0, 4, 8]], axis=1))
        dens = np.array(counts) / np.maximum(vol, 1e-30)
        self.edge_estimate = int(np.sum(np.array(counts) * np.maximum(48.0, 1.6 * dens * 4.0 / 3.0 * math.pi * 125.0)))


def read_timing(model: "Model") -> dict:
    """Per-phase totals since timing was enabled: {name: (ms, calls)}."""
    t = TimingC()
    _check(lib.mpip_timing_read(model._h, ctypes.byref(t)))
    return {t.name[k].value.decode(): (float(t.ms[k]), int(t.calls[k])) for k in range(t.n)}


def workspace_status(model: "Model", stream=None) -> int:
    """Synchronise and return the status code of the model's workspace."""
    ne = ctypes.c_int64()
    sp = _stream_ptr(model.torch, model.device, stream)
    return int(lib.mpip_workspace_status(ctypes.c_void_p(model._ws.data_ptr()), ctypes.c_void_p(sp),
                                         ctypes.byref(ne)))


def evaluate_batch(model: "Model", batch: Batch, K=None, precision="fp32", max_edges=None, stream=None,
                   check: bool = True):
    """Energies [B], forces [N,3], virials [B,3,3] of a Batch (cuda tensors)."""
    torch = model.torch
    K = model.hp.n_layers if K is None else int(K)
    prec = PRECISIONS[precision]
    if max_edges is None:
        max_edges = batch.edge_estimate
    for attempt in range(2):
        nb = ctypes.c_size_t()
        _check(lib.mpip_batch_workspace_size(model._h, batch.n_atoms, batch.B, prec, K, max_edges, ctypes.byref(nb)))
        if model._ws is None or model._ws.numel() < nb.value:
            model._ws = None
            model._ws = torch.empty(nb.value, dtype=torch.uint8, device=model.device)
        ws = model._ws
        o = {"energy": torch.empty(batch.B, dtype=torch.float64, device=model.device),
             "forces": torch.empty((batch.n_atoms, 3), dtype=torch.float64, device=model.device),
             "virial": torch.empty((batch.B, 3, 3), dtype=torch.float64, device=model.device)}
        sp = _stream_ptr(torch, model.device, stream)
        _check(lib.mpip_evaluate_batch(
            model._h, batch.B, batch.atom_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ctypes.c_void_p(batch.positions.data_ptr()), ctypes.c_void_p(batch.species.data_ptr()),
            batch.cells.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            batch.pbc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), prec, K, ctypes.c_void_p(sp),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), max_edges, ctypes.c_void_p(o["energy"].data_ptr()),
            ctypes.c_void_p(o["forces"].data_ptr()), ctypes.c_void_p(o["virial"].data_ptr())))
        if not check:
            return o
        ne = ctypes.c_int64()
        st = lib.mpip_workspace_status(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(sp), ctypes.byref(ne))
        if st == ECAPACITY and attempt == 0:
            max_edges = int(ne.value * 1.05) + 1024
            continue
        _check(st)
        o["n_edges"] = int(ne.value)
        return o
    raise MpipError(ECAPACITY, "edge capacity")


def neighbor_list(positions, cell, pbc, r_cut: float, capacity: Optional[int] = None, stream=None):
    """Edges (i, j, S) in input indices as cuda int32 tensors (unordered)."""
    import torch
    dev = positions.device
    N = int(positions.shape[0])
    species = torch.zeros(N, dtype=torch.int32, device=dev)
    if capacity is None:
        capacity = estimate_edges(N, cell, r_cut)
    for attempt in range(2):
        nbytes = int(lib.mpip_neighbor_workspace_size(N, capacity))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        ei = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        ej = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        es = torch.empty((max(capacity, 1), 3), dtype=torch.int32, device=dev)
        sysc = _system(positions, species, cell, pbc, None)
        ne = ctypes.c_int64()
        sp = _stream_ptr(torch, dev, stream)
        st = lib.mpip_neighbor_list(ctypes.byref(sysc), float(r_cut), ctypes.c_void_p(sp),
                                    ctypes.c_void_p(ws.data_ptr()), nbytes, capacity, ctypes.c_void_p(ei.data_ptr()),
                                    ctypes.c_void_p(ej.data_ptr()), ctypes.c_void_p(es.data_ptr()), ctypes.byref(ne))
        if st == ECAPACITY and attempt == 0 and ne.value > capacity:
            capacity = int(ne.value) + 16
            continue
        _check(st)
        n = int(ne.value)
        return ei[:n], ej[:n], es[:n]
    raise MpipError(ECAPACITY, "edge capacity")


def slab_share(positions, species, cell, n_parts: int, part: int, halo: float, axis: int = 0,
               capacity: Optional[int] = None, stream=None):
    """One slab partition with its halo, built on the GPU.  Returns
    (positions [n,3] f64, species [n] i32, input index [n] i32, n_owned) as
    cuda tensors; root atoms first.  Evaluate it with pbc[axis] = False."""
    import torch
    dev = positions.device
    N = int(positions.shape[0])
    c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    Lax = float(c[4 * axis])
    if capacity is None:
        capacity = int(N / n_parts + 2 * N * halo / Lax) + 1024
    for attempt in range(2):
        nbytes = int(lib.mpip_slab_workspace_size(N, Lax, float(halo)))
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        op = torch.empty((capacity, 3), dtype=torch.float64, device=dev)
        osp = torch.empty(capacity, dtype=torch.int32, device=dev)
        oix = torch.empty(capacity, dtype=torch.int32, device=dev)
        nl, no = ctypes.c_int64(), ctypes.c_int64()
        st = lib.mpip_slab_share(ctypes.c_void_p(positions.data_ptr()), ctypes.c_void_p(species.data_ptr()), N,
                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), axis, n_parts, part,
                                 float(halo), ctypes.c_void_p(_stream_ptr(torch, dev, stream)),
                                 ctypes.c_void_p(ws.data_ptr()), nbytes, capacity, ctypes.c_void_p(op.data_ptr()),
                                 ctypes.c_void_p(osp.data_ptr()), ctypes.c_void_p(oix.data_ptr()),
                                 ctypes.byref(nl), ctypes.byref(no))
        if st == ECAPACITY and attempt == 0 and nl.value > capacity:
            capacity = int(nl.value)
            continue
        _check(st)
        n = int(nl.value)
        return op[:n], osp[:n], oix[:n], int(no.value)
    raise MpipError(ECAPACITY, "share capacity")


def bfs_share(positions, species, cell, n_parts: int, part: int, K: int, r_cut: float, axis: int = 0,
              pbc=(True, True, True), capacity: Optional[int] = None, max_edges: Optional[int] = None,
              stream=None):
    """One slab partition with a graph halo (atoms within K hops of a root),
    built on the GPU.  Returns (positions [n,3] f64, species [n] i32, input
    index [n] i32, n_owned) as cuda tensors; root atoms first.  Evaluate it
    with pbc[axis] = False."""
    import torch
    dev = positions.device
    N = int(positions.shape[0])
    c = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    Lax = float(c[axis, axis])
    if capacity is None:
        capacity = int(N / n_parts + 2 * N * K * r_cut / Lax) + 1024
    if max_edges is None:
        max_edges = estimate_edges(N, cell, r_cut)
    sysc = _system(positions, species, cell, pbc, None)
    for attempt in range(2):
        nbytes = int(lib.mpip_bfs_share_workspace_size(N, Lax, int(K), float(r_cut), max_edges))
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        op = torch.empty((capacity, 3), dtype=torch.float64, device=dev)
        osp = torch.empty(capacity, dtype=torch.int32, device=dev)
        oix = torch.empty(capacity, dtype=torch.int32, device=dev)
        nl, no, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        st = lib.mpip_bfs_share(ctypes.byref(sysc), float(r_cut), axis, n_parts, part, int(K),
                                ctypes.c_void_p(_stream_ptr(torch, dev, stream)), ctypes.c_void_p(ws.data_ptr()),
                                nbytes, max_edges, capacity, ctypes.c_void_p(op.data_ptr()),
                                ctypes.c_void_p(osp.data_ptr()), ctypes.c_void_p(oix.data_ptr()),
                                ctypes.byref(nl), ctypes.byref(no), ctypes.byref(ne))
        if st == ECAPACITY and attempt == 0:
            capacity = max(capacity, int(nl.value))
            max_edges = max(max_edges, int(ne.value * 1.05) + 1024)
            continue
        _check(st)
        n = int(nl.value)
        return op[:n], osp[:n], oix[:n], int(no.value)
    raise MpipError(ECAPACITY, "share capacity")


def accumulate_rows(src, index, dst, stream=None):
    """dst[index[k]] += src[k] (rows of 3 doubles) on the GPU."""
    import torch
    _check(lib.mpip_accumulate_rows(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(index.data_ptr()),
                                    int(src.shape[0]), int(dst.shape[0]), ctypes.c_void_p(dst.data_ptr()),
                                    ctypes.c_void_p(_stream_ptr(torch, dst.device, stream))))


def _autograd():
    import torch

    class MPIPEnergy(torch.autograd.Function):
        """E(positions) with the library's hand-written adjoint as backward:
        forward runs one full evaluation (energy, forces, virial); backward
        returns -grad_E * F for the positions (no second GPU pass).  The
        virial is returned as a second, non-differentiable output."""

        @staticmethod
        def forward(ctx, positions, model, species, cell, pbc, K, precision, n_owned):
            o = model.evaluate(positions.detach(), species, cell, pbc, K=K, precision=precision,
                               n_owned=n_owned)
            ctx.save_for_backward(o["forces"])
            ctx.mark_non_differentiable(o["virial"])
            return o["energy"][0], o["virial"]

        @staticmethod
        def backward(ctx, g_energy, g_virial):
            (F,) = ctx.saved_tensors
            return -g_energy * F, None, None, None, None, None, None, None

    return MPIPEnergy


_MPIPEnergy = None


def MPIPEnergy():
    """The torch.autograd.Function class (created lazily, needs torch)."""
    global _MPIPEnergy
    if _MPIPEnergy is None:
        _MPIPEnergy = _autograd()
    return _MPIPEnergy


def energy(positions, model: Model, species, cell, pbc=(True, True, True), K=None, precision="fp32",
           n_owned=None):
    """Differentiable energy: E, W = energy(...); E.backward() gives
    positions.grad = -F."""
    return MPIPEnergy().apply(positions, model, species, cell, pbc, K, precision, n_owned)
