"""ctypes binding of include/ace.h (argument marshalling only).

Every step of the ACE build runs in the HIP library; this module only turns
torch tensors into device pointers and the current torch stream into the
hipStream_t argument.  It fails loudly when the library is missing: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacex.so")

ACE_OK, ACE_ERR_ARG, ACE_ERR_SIZE, ACE_ERR_WORKSPACE, ACE_ERR_HIP, ACE_ERR_NODEV = range(6)
ACE_FP64, ACE_FP32 = 0, 1
N_STAGES = 10
STAGE_NAMES = ["yz_fwd", "x_poisson", "yz_inv", "w_accumulate", "m_product", "cholesky_inv",
               "xi_product", "small", "apply_products", "x_energy"]
EXPORTS = ["ace_plan_create", "ace_plan_destroy", "ace_workspace_bytes",
           "ace_apply_workspace_bytes", "ace_build", "ace_apply", "exx_energy",
           "ace_error_string", "ace_last_hip_error", "ace_set_profiling", "ace_profile_read",
           "ace_plan_set_tiling", "ace_plan_tiling", "ace_plan_set_schedule", "ace_plan_schedule", "ace_overlap_integrals", "ace_wannier", "ace_mlp_screen",
           "ace_mlp_weight_count", "ace_batch_create", "ace_batch_destroy",
           "ace_batch_workspace_bytes", "ace_batch_build", "ace_batch_lanes", "scdm_workspace_bytes",
           "scdm_preselect", "scdm_localize", "ace_apply_noalloc", "ace_screen_mask",
           "ace_screen_mask_host"]
PROBE_EXPORTS = ["ace_bandwidth_probe"]
PROBE_KINDS = {"read_write": 0, "read": 1, "write": 2}
ACE_BATCH_MAX = 1024
ACE_BATCH_EAGER = 1
ACE_BATCH_NO_LANES = 2


class AceError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = "%s failed: %s" % (where, _error_string(code))
        if code == ACE_ERR_HIP:
            msg += " (hipError %d)" % _LIB.ace_last_hip_error()
        super().__init__(msg)


class ScreenDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rho_cut", ctypes.c_double), ("budget", ctypes.c_double),
                ("safety", ctypes.c_double), ("mlp_weights", ctypes.c_void_p)]


class ScreenReport(ctypes.Structure):
    _fields_ = [("pairs_kept", ctypes.c_int64), ("pairs_total", ctypes.c_int64),
                ("predicted_skipped", ctypes.c_double), ("fallback", ctypes.c_int)]


ACE_SCREEN_OVERLAP, ACE_SCREEN_MLP = 0, 1


class AceDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("cell", ctypes.c_double * 3), ("n_orb", ctypes.c_int),
                ("precision", ctypes.c_int), ("alpha", ctypes.c_double)]


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libacex.so (built in-tree by build.py); raise if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError("libacex.so is not built (%s); run __graft_entry__.build()" % path)
    # torch first: the library must bind to the HIP runtime torch has loaded,
    # or the process ends up with two runtimes that do not share devices
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, sz, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    lib.ace_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(AceDesc)]
    lib.ace_plan_create.restype = i
    lib.ace_plan_destroy.argtypes = [vp]
    lib.ace_plan_destroy.restype = None
    lib.ace_workspace_bytes.argtypes = [vp]
    lib.ace_workspace_bytes.restype = sz
    lib.ace_apply_workspace_bytes.argtypes = [vp, i]
    lib.ace_apply_workspace_bytes.restype = sz
    lib.ace_build.argtypes = [vp, vp, vp, sz, vp, vp, vp, vp, vp, vp, vp]
    lib.ace_build.restype = i
    lib.ace_apply.argtypes = [vp, vp, vp, sz, vp, vp, i, vp]
    lib.ace_apply.restype = i
    lib.exx_energy.argtypes = [vp, vp, vp, sz, vp, vp, vp, vp]
    lib.exx_energy.restype = i
    lib.ace_error_string.argtypes = [i]
    lib.ace_error_string.restype = ctypes.c_char_p
    lib.ace_last_hip_error.argtypes = []
    lib.ace_last_hip_error.restype = i
    lib.ace_set_profiling.argtypes = [vp, i]
    lib.ace_set_profiling.restype = i
    lib.ace_profile_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i)]
    lib.ace_profile_read.restype = i
    lib.ace_plan_set_tiling.argtypes = [vp, i, i, i]
    lib.ace_plan_set_tiling.restype = i
    lib.ace_plan_tiling.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.ace_plan_tiling.restype = i
    lib.ace_plan_schedule.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.ace_plan_schedule.restype = i
    lib.ace_plan_set_schedule.argtypes = [vp, i]
    lib.ace_plan_set_schedule.restype = i
    lib.ace_overlap_integrals.argtypes = [vp, vp, vp, sz, vp, vp]
    lib.ace_overlap_integrals.restype = i
    lib.ace_wannier.argtypes = [vp, vp, vp, vp, vp]
    lib.ace_wannier.restype = i
    lib.ace_mlp_screen.argtypes = [vp, vp, vp, vp, vp]
    lib.ace_mlp_screen.restype = i
    lib.ace_mlp_weight_count.argtypes = []
    lib.ace_mlp_weight_count.restype = i
    lib.ace_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i]
    lib.ace_batch_create.restype = i
    lib.ace_batch_destroy.argtypes = [vp]
    lib.ace_batch_destroy.restype = None
    lib.ace_batch_workspace_bytes.argtypes = [vp]
    lib.ace_batch_workspace_bytes.restype = sz
    lib.ace_batch_build.argtypes = [vp, vp, vp, sz, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, i]
    lib.ace_batch_build.restype = i
    lib.ace_batch_lanes.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]
    lib.ace_batch_lanes.restype = i
    lib.scdm_workspace_bytes.argtypes = [vp, i]
    lib.scdm_workspace_bytes.restype = sz
    lib.scdm_preselect.argtypes = [vp, vp, vp, sz, vp, vp, vp]
    lib.scdm_preselect.restype = i
    lib.scdm_localize.argtypes = [vp, vp, vp, sz, vp, vp, i, vp, vp, vp]
    lib.scdm_localize.restype = i
    lib.ace_screen_mask.argtypes = [vp, vp, vp, sz, vp, ctypes.POINTER(ScreenDesc), vp,
                                    ctypes.POINTER(ScreenReport)]
    lib.ace_screen_mask.restype = i
    lib.ace_screen_mask_host.argtypes = [i, ctypes.POINTER(ScreenDesc), vp, vp, vp,
                                         ctypes.POINTER(ScreenReport)]
    lib.ace_screen_mask_host.restype = i
    lib.ace_apply_noalloc.argtypes = [vp, vp, vp, vp, i, vp]
    lib.ace_apply_noalloc.restype = i
    lib.ace_bandwidth_probe.argtypes = [i, vp, vp, sz, i]
    lib.ace_bandwidth_probe.restype = i
    _LIB = lib
    return lib


def _error_string(code: int) -> str:
    return load().ace_error_string(code).decode()


def _check(code: int, where: str):
    if code != ACE_OK:
        raise AceError(code, where)


def _ptr(t) -> int:
    """Device (or host) address of a torch tensor, None -> 0."""
    if t is None:
        return 0
    return int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _mask_buffer(mask, n_orb: int):
    if mask is None:
        return None, 0
    m = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
    if m.shape != (n_orb, n_orb):
        raise ValueError("pair_mask must be (%d, %d)" % (n_orb, n_orb))
    return m, m.ctypes.data


def _tensor(t, name: str, shape=None, dtype: str = "float64", device=None, min_bytes: int = 0,
            cuda: bool = True):
    """Check that t is a contiguous device tensor of the given dtype and shape
    (and on `device`) before its address reaches a kernel: the C-ABI sees
    only pointers, so a wrong size or a host tensor would be read or written
    out of bounds on the GPU.  Raises ValueError."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor, got %s" % (name, type(t).__name__))
    if dtype is not None and t.dtype != getattr(torch, dtype):
        raise ValueError("%s must be %s (is %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (has %s)" % (name, tuple(shape), tuple(t.shape)))
    if t.numel() * t.element_size() < min_bytes:
        raise ValueError("%s holds %d bytes, the call needs %d"
                         % (name, t.numel() * t.element_size(), min_bytes))
    if cuda:
        _on_device(device, (name, t))
    return t


def _on_device(device, *named):
    """Every (name, tensor) is a device tensor, on `device` (default: the
    first one's) and on the current device."""
    import torch
    for name, t in named:
        if not t.is_cuda:
            raise ValueError("%s must be a device tensor (is on %s)" % (name, t.device))
        if device is None:
            device = t.device
        if t.device != device:
            raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
        if t.device.index != torch.cuda.current_device():
            raise ValueError("%s is on %s but the current device is cuda:%d"
                             % (name, t.device, torch.cuda.current_device()))


class Plan:
    """A host-only ACE plan (grid, cell, orbital count, precision, alpha)."""

    def __init__(self, n: int, cell: Sequence[float], n_orb: int, precision: str = "fp64",
                 alpha: float = 0.25, grid: Optional[Sequence[int]] = None):
        lib = load()
        d = AceDesc()
        g = list(grid) if grid is not None else [n, n, n]
        for a in range(3):
            d.n[a] = int(g[a])
        cl = list(cell) if np.ndim(cell) == 1 else [float(cell[a][a]) for a in range(3)]
        for a in range(3):
            d.cell[a] = float(cl[a])
        d.n_orb = int(n_orb)
        d.precision = {"fp64": ACE_FP64, "fp32": ACE_FP32}[precision] if isinstance(precision, str) else int(precision)
        d.alpha = float(alpha)
        h = ctypes.c_void_p()
        _check(lib.ace_plan_create(ctypes.byref(h), ctypes.byref(d)), "ace_plan_create")
        self._h = h
        self.n, self.cell, self.n_orb, self.alpha = g[0], cl, int(n_orb), float(alpha)
        self.grid = tuple(int(v) for v in g)
        self.precision = d.precision
        self.npts = g[0] * g[1] * g[2]
        blk, ch, pen = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.ace_plan_tiling(h, ctypes.byref(blk), ctypes.byref(ch), ctypes.byref(pen)),
               "ace_plan_tiling")
        self.tiling = (blk.value, ch.value, pen.value)
        self.four_pass = False

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.ace_plan_destroy(self._h)
            self._h = None

    def workspace_bytes(self) -> int:
        return int(load().ace_workspace_bytes(self._h))

    def apply_workspace_bytes(self, n_vec: int) -> int:
        return int(load().ace_apply_workspace_bytes(self._h, int(n_vec)))

    def orbital_shape(self, count: Optional[int] = None):
        return (self.n_orb if count is None else int(count),) + self.grid

    def check_orbitals(self, t, name: str = "phi", count: Optional[int] = None, device=None,
                       cuda: bool = True):
        """Validate an orbital-major float64 (device) tensor for this plan."""
        return _tensor(t, name, self.orbital_shape(count), device=device, cuda=cuda)

    def set_tiling(self, block: int, chunk: int = 0, pencils: int = 0):
        _check(load().ace_plan_set_tiling(self._h, int(block), int(chunk), int(pencils)),
               "ace_plan_set_tiling")
        self.tiling = (int(block), int(chunk), int(pencils))

    def set_schedule(self, four_pass: bool):
        """Four transform passes everywhere (True) or three where they apply (False)."""
        _check(load().ace_plan_set_schedule(self._h, 1 if four_pass else 0),
               "ace_plan_set_schedule")
        self.four_pass = bool(four_pass)

    def schedule(self):
        """(full-tile schedule: "three_pass", "rows_fused" or "four_pass",
        whether a (y, z) plane fits LDS) for the current shape."""
        kind, plane = ctypes.c_int(), ctypes.c_int()
        _check(load().ace_plan_schedule(self._h, ctypes.byref(kind), ctypes.byref(plane)),
               "ace_plan_schedule")
        return ["three_pass", "rows_fused", "four_pass"][kind.value], bool(plane.value)

    def set_profiling(self, on: bool):
        _check(load().ace_set_profiling(self._h, 1 if on else 0), "ace_set_profiling")

    def profile_read(self):
        ms = (ctypes.c_double * N_STAGES)()
        cnt = (ctypes.c_int * N_STAGES)()
        _check(load().ace_profile_read(self._h, ms, cnt), "ace_profile_read")
        return {STAGE_NAMES[i]: (ms[i], cnt[i]) for i in range(N_STAGES)}


def workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def build_into(plan: Plan, phi, W, M, xi, ex, info, ws, pair_mask=None, stream=None):
    """ace_build on caller-provided torch tensors (no allocation)."""
    plan.check_orbitals(phi, cuda=False)
    plan.check_orbitals(W, "W", cuda=False)
    plan.check_orbitals(xi, "xi", cuda=False)
    _tensor(M, "M", (plan.n_orb, plan.n_orb), cuda=False)
    _tensor(ex, "ex", None, min_bytes=8, cuda=False)
    _tensor(info, "info", None, "int32", min_bytes=4, cuda=False)
    _tensor(ws, "ws", None, None, min_bytes=plan.workspace_bytes(), cuda=False)
    _on_device(None, ("phi", phi), ("W", W), ("xi", xi), ("M", M), ("ex", ex), ("info", info),
               ("ws", ws))
    m, mptr = _mask_buffer(pair_mask, plan.n_orb)
    rc = load().ace_build(plan.handle, _stream(stream), _ptr(ws), ws.numel() * ws.element_size(),
                          _ptr(phi), mptr or None, _ptr(W), _ptr(M), _ptr(xi), _ptr(ex), _ptr(info))
    _check(rc, "ace_build")


def ace_build(plan: Plan, phi, pair_mask=None, ws=None, stream=None):
    """W, M, xi, ex, info as torch tensors on phi's device."""
    import torch
    plan.check_orbitals(phi)
    dev = phi.device
    k = plan.n_orb
    W = torch.empty_like(phi)
    xi = torch.empty_like(phi)
    M = torch.empty((k, k), dtype=torch.float64, device=dev)
    ex = torch.zeros((1,), dtype=torch.float64, device=dev)
    info = torch.zeros((1,), dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(plan.workspace_bytes(), dev)
    build_into(plan, phi, W, M, xi, ex, info, ws, pair_mask, stream)
    return {"W": W, "M": M, "xi": xi, "ex": ex, "info": info}


def apply_into(plan: Plan, xi, psi, out, ws, stream=None):
    plan.check_orbitals(xi, "xi", cuda=False)
    if not hasattr(psi, "shape") or psi.dim() != 4:
        raise ValueError("psi must be a (n_vec, n1, n2, n3) tensor")
    n_vec = int(psi.shape[0])
    if n_vec < 1:
        raise ValueError("psi holds no vectors")
    plan.check_orbitals(psi, "psi", count=n_vec, cuda=False)
    plan.check_orbitals(out, "out", count=n_vec, cuda=False)
    _tensor(ws, "ws", None, None, min_bytes=plan.apply_workspace_bytes(n_vec), cuda=False)
    _on_device(None, ("xi", xi), ("psi", psi), ("out", out), ("ws", ws))
    rc = load().ace_apply(plan.handle, _stream(stream), _ptr(ws), ws.numel() * ws.element_size(),
                          _ptr(xi), _ptr(psi), n_vec, _ptr(out))
    _check(rc, "ace_apply")


def apply_noalloc_into(plan: Plan, xi, psi, out, stream=None):
    """ace_apply_noalloc: the apply with the library's static scratch (no
    workspace, no allocation in the library)."""
    plan.check_orbitals(xi, "xi", cuda=False)
    if not hasattr(psi, "shape") or psi.dim() != 4 or int(psi.shape[0]) < 1:
        raise ValueError("psi must be a (n_vec, n1, n2, n3) tensor")
    n_vec = int(psi.shape[0])
    plan.check_orbitals(psi, "psi", count=n_vec, cuda=False)
    plan.check_orbitals(out, "out", count=n_vec, cuda=False)
    _on_device(None, ("xi", xi), ("psi", psi), ("out", out))
    rc = load().ace_apply_noalloc(plan.handle, _stream(stream), _ptr(xi), _ptr(psi), n_vec,
                                  _ptr(out))
    _check(rc, "ace_apply_noalloc")


def ace_apply(plan: Plan, xi, psi, ws=None, stream=None):
    import torch
    plan.check_orbitals(xi, "xi", cuda=False)
    if not hasattr(psi, "shape") or psi.dim() != 4:
        raise ValueError("psi must be a (n_vec, n1, n2, n3) tensor")
    plan.check_orbitals(psi, "psi", count=int(psi.shape[0]), cuda=False)
    _on_device(None, ("xi", xi), ("psi", psi))
    out = torch.empty_like(psi)
    if ws is None:
        ws = workspace(plan.apply_workspace_bytes(int(psi.shape[0])), psi.device)
    apply_into(plan, xi, psi, out, ws, stream)
    return out


def exx_energy(plan: Plan, phi, pair_mask=None, pair_energies: bool = False, ws=None, stream=None):
    """(ex tensor[1], pair_e tensor[n_orb, n_orb] or None)."""
    import torch
    plan.check_orbitals(phi)
    dev = phi.device
    ex = torch.zeros((1,), dtype=torch.float64, device=dev)
    pe = torch.zeros((plan.n_orb, plan.n_orb), dtype=torch.float64, device=dev) if pair_energies else None
    if ws is None:
        ws = workspace(plan.workspace_bytes(), dev)
    _tensor(ws, "ws", None, None, device=dev, min_bytes=plan.workspace_bytes())
    m, mptr = _mask_buffer(pair_mask, plan.n_orb)
    rc = load().exx_energy(plan.handle, _stream(stream), _ptr(ws), ws.numel() * ws.element_size(),
                           _ptr(phi), mptr or None, _ptr(ex), _ptr(pe))
    _check(rc, "exx_energy")
    return ex, pe


# ------------------------------------------------------------------ pair screening

def overlap_integrals(plan: Plan, phi, ws=None, stream=None):
    """S[i, j] = dV sum_r |phi_i| |phi_j| (device float64 [n_orb, n_orb])."""
    import torch
    plan.check_orbitals(phi)
    S = torch.empty((plan.n_orb, plan.n_orb), dtype=torch.float64, device=phi.device)
    if ws is None:
        ws = workspace(plan.workspace_bytes(), phi.device)
    _tensor(ws, "ws", None, None, device=phi.device, min_bytes=plan.workspace_bytes())
    rc = load().ace_overlap_integrals(plan.handle, _stream(stream), _ptr(ws),
                                      ws.numel() * ws.element_size(), _ptr(phi), _ptr(S))
    _check(rc, "ace_overlap_integrals")
    return S


def wannier(plan: Plan, phi, stream=None):
    """(z [n_orb, 6], feat [n_orb, 4]) device float64: Berry-phase moments and
    (centre xyz, spread) of each orbital density."""
    import torch
    plan.check_orbitals(phi)
    z = torch.empty((plan.n_orb, 6), dtype=torch.float64, device=phi.device)
    feat = torch.empty((plan.n_orb, 4), dtype=torch.float64, device=phi.device)
    rc = load().ace_wannier(plan.handle, _stream(stream), _ptr(phi), _ptr(z), _ptr(feat))
    _check(rc, "ace_wannier")
    return z, feat


def mlp_weight_count() -> int:
    return int(load().ace_mlp_weight_count())


def mlp_screen(plan: Plan, feat, weights, stream=None):
    """pred [n_orb, n_orb] device float32: predicted log10 |e_ij| for i <= j
    (entries below the diagonal are NaN)."""
    import torch
    _tensor(feat, "feat", (plan.n_orb, 4))
    w = weights if hasattr(weights, "data_ptr") else torch.from_numpy(
        np.ascontiguousarray(weights, dtype=np.float32)).to(feat.device)
    _tensor(w, "weights", (mlp_weight_count(),), "float32", device=feat.device)
    pred = torch.full((plan.n_orb, plan.n_orb), float("nan"), dtype=torch.float32,
                      device=feat.device)
    rc = load().ace_mlp_screen(plan.handle, _stream(stream), _ptr(feat), _ptr(w), _ptr(pred))
    _check(rc, "ace_mlp_screen")
    return pred


def _screen_desc(kind: str, rho_cut: float, budget: float, safety: float, weights):
    d = ScreenDesc()
    d.kind = {"overlap": ACE_SCREEN_OVERLAP, "mlp": ACE_SCREEN_MLP}[kind]
    d.rho_cut, d.budget, d.safety = float(rho_cut), float(budget), float(safety)
    d.mlp_weights = _ptr(weights) if weights is not None else None
    return d


def _report(rep: ScreenReport):
    return {"pairs_kept": int(rep.pairs_kept), "pairs_total": int(rep.pairs_total),
            "predicted_skipped": float(rep.predicted_skipped), "fallback": bool(rep.fallback)}


def screen_mask(plan: Plan, phi, kind: str, rho_cut: float = 0.0, budget: float = 0.0,
                safety: float = 2.0, weights=None, ws=None, stream=None):
    """ace_screen_mask: (host uint8 [n_orb, n_orb] pair mask, report dict)."""
    plan.check_orbitals(phi)
    if weights is not None:
        _tensor(weights, "weights", (mlp_weight_count(),), "float32", device=phi.device)
    if ws is None:
        ws = workspace(plan.workspace_bytes(), phi.device)
    _tensor(ws, "ws", None, None, device=phi.device, min_bytes=plan.workspace_bytes())
    mask = np.zeros((plan.n_orb, plan.n_orb), dtype=np.uint8)
    rep = ScreenReport()
    d = _screen_desc(kind, rho_cut, budget, safety, weights)
    rc = load().ace_screen_mask(plan.handle, _stream(stream), _ptr(ws),
                                ws.numel() * ws.element_size(), _ptr(phi), ctypes.byref(d),
                                mask.ctypes.data, ctypes.byref(rep))
    _check(rc, "ace_screen_mask")
    return mask, _report(rep)


def screen_mask_host(kind: str, S=None, pred=None, rho_cut: float = 0.0, budget: float = 0.0,
                     safety: float = 2.0):
    """ace_screen_mask_host on host arrays (no device)."""
    n = int((S if S is not None else pred).shape[0])
    Sa = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
    Pa = None if pred is None else np.ascontiguousarray(pred, dtype=np.float32)
    for a in (Sa, Pa):
        if a is not None and a.shape != (n, n):
            raise ValueError("screening inputs must be (n, n)")
    mask = np.zeros((n, n), dtype=np.uint8)
    rep = ScreenReport()
    d = _screen_desc(kind, rho_cut, budget, safety, None)
    rc = load().ace_screen_mask_host(n, ctypes.byref(d), None if Sa is None else Sa.ctypes.data,
                                     None if Pa is None else Pa.ctypes.data, mask.ctypes.data,
                                     ctypes.byref(rep))
    _check(rc, "ace_screen_mask_host")
    return mask, _report(rep)


# ------------------------------------------------------------------ batches

def _ptr_array(items):
    arr = (ctypes.c_void_p * len(items))()
    for k, t in enumerate(items):
        arr[k] = _ptr(t) if t is not None else None
    return arr


class Batch:
    """Independent systems built together (ace_batch_*): one recorded HIP
    graph whose branches run the instances concurrently."""

    def __init__(self, plans: Sequence[Plan], pair_masks=None):
        lib = load()
        self.plans = list(plans)
        n = len(self.plans)
        hs = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        masks = None
        keep = []
        if pair_masks is not None:
            masks = (ctypes.c_void_p * n)()
            for k, (p, m) in enumerate(zip(self.plans, pair_masks)):
                buf, ptr = _mask_buffer(m, p.n_orb)
                keep.append(buf)
                masks[k] = ptr or None
        h = ctypes.c_void_p()
        _check(lib.ace_batch_create(ctypes.byref(h), hs, masks, n), "ace_batch_create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.ace_batch_destroy(self._h)
            self._h = None

    def workspace_bytes(self) -> int:
        return int(load().ace_batch_workspace_bytes(self._h))

    def lanes(self):
        """(lanes, tiles in the shared pass launches, tiles on the single-system kernels)."""
        n = ctypes.c_int()
        bt, ot = ctypes.c_int64(), ctypes.c_int64()
        _check(load().ace_batch_lanes(self._h, ctypes.byref(n), ctypes.byref(bt), ctypes.byref(ot)),
               "ace_batch_lanes")
        return n.value, bt.value, ot.value

    def outputs(self, phis):
        """Fresh W, M, xi lists and ex[count], info[count] for phis."""
        import torch
        dev = phis[0].device
        W = [torch.empty_like(p) for p in phis]
        xi = [torch.empty_like(p) for p in phis]
        M = [torch.empty((pl.n_orb, pl.n_orb), dtype=torch.float64, device=dev)
             for pl in self.plans]
        ex = torch.zeros((len(phis),), dtype=torch.float64, device=dev)
        info = torch.zeros((len(phis),), dtype=torch.int32, device=dev)
        return {"W": W, "M": M, "xi": xi, "ex": ex, "info": info}

    def build_into(self, phis, out, ws, eager: bool = False, stream=None, lanes: bool = True):
        if len(phis) != len(self.plans):
            raise ValueError("expected %d orbital sets" % len(self.plans))
        for key in ("W", "M", "xi"):
            if len(out[key]) != len(self.plans):
                raise ValueError("expected %d %s tensors" % (len(self.plans), key))
        named = []
        for k, p in enumerate(self.plans):
            for key, t in (("phis", phis[k]), ("W", out["W"][k]), ("xi", out["xi"][k])):
                p.check_orbitals(t, "%s[%d]" % (key, k), cuda=False)
                named.append(("%s[%d]" % (key, k), t))
            _tensor(out["M"][k], "M[%d]" % k, (p.n_orb, p.n_orb), cuda=False)
            named.append(("M[%d]" % k, out["M"][k]))
        _tensor(out["ex"], "ex", (len(self.plans),), cuda=False)
        _tensor(out["info"], "info", (len(self.plans),), "int32", cuda=False)
        _tensor(ws, "ws", None, None, min_bytes=self.workspace_bytes(), cuda=False)
        _on_device(None, *named, ("ex", out["ex"]), ("info", out["info"]), ("ws", ws))
        rc = load().ace_batch_build(self._h, _stream(stream), _ptr(ws),
                                    ws.numel() * ws.element_size(), _ptr_array(phis),
                                    _ptr_array(out["W"]), _ptr_array(out["M"]),
                                    _ptr_array(out["xi"]), _ptr(out["ex"]), _ptr(out["info"]),
                                    (ACE_BATCH_EAGER if eager else 0) |
                                    (0 if lanes else ACE_BATCH_NO_LANES))
        _check(rc, "ace_batch_build")

    def build(self, phis, ws=None, eager: bool = False, stream=None, lanes: bool = True):
        out = self.outputs(phis)
        if ws is None:
            ws = workspace(self.workspace_bytes(), phis[0].device)
        self.build_into(phis, out, ws, eager, stream, lanes)
        return out


# ------------------------------------------------------------------ SCDM localisation

def scdm_preselect(plan: Plan, phi, ws=None, stream=None):
    """Kept grid points of the s' rule (device int32 tensor, increasing)."""
    import torch
    plan.check_orbitals(phi)
    if ws is None:
        ws = workspace(int(load().scdm_workspace_bytes(plan.handle, 0)), phi.device)
    _tensor(ws, "ws", None, None, device=phi.device,
            min_bytes=int(load().scdm_workspace_bytes(plan.handle, 0)))
    points = torch.empty((plan.npts,), dtype=torch.int32, device=phi.device)
    count = torch.zeros((1,), dtype=torch.int32, device=phi.device)
    rc = load().scdm_preselect(plan.handle, _stream(stream), _ptr(ws),
                               ws.numel() * ws.element_size(), _ptr(phi), _ptr(points),
                               _ptr(count))
    _check(rc, "scdm_preselect")
    m = int(count.item())
    return points[:m]


def scdm_localize(plan: Plan, phi, points=None, ws=None, stream=None):
    """(pivots [n_orb] int32, phi_loc like phi, info [1] int32) on the device;
    points None: every grid point."""
    import torch
    plan.check_orbitals(phi)
    m = plan.npts if points is None else int(points.numel())
    if points is not None:
        _tensor(points, "points", (m,), "int32", device=phi.device)
    if ws is None:
        ws = workspace(int(load().scdm_workspace_bytes(plan.handle, m)), phi.device)
    _tensor(ws, "ws", None, None, device=phi.device,
            min_bytes=int(load().scdm_workspace_bytes(plan.handle, m)))
    pivots = torch.empty((plan.n_orb,), dtype=torch.int32, device=phi.device)
    loc = torch.empty_like(phi)
    info = torch.zeros((1,), dtype=torch.int32, device=phi.device)
    rc = load().scdm_localize(plan.handle, _stream(stream), _ptr(ws),
                              ws.numel() * ws.element_size(), _ptr(phi), _ptr(points), m,
                              _ptr(pivots), _ptr(loc), _ptr(info))
    _check(rc, "scdm_localize")
    return pivots, loc, info


def scdm(plan: Plan, phi, preselect: bool = True, stream=None):
    """SCDM localisation with (default) or without the s' preselection."""
    pts = scdm_preselect(plan, phi, stream=stream) if preselect else None
    pivots, loc, info = scdm_localize(plan, phi, pts, stream=stream)
    return {"points": pts, "pivots": pivots, "phi_loc": loc, "info": info}


# ------------------------------------------------------------------ bandwidth probes

def bandwidth_probe(kind: str, buf, blocks: int, stream=None):
    """One streaming launch over the device tensor `buf` (include/ace_probe.h):
    kind 'read_write' (in place), 'read' or 'write'."""
    _tensor(buf, "buf", None, None, min_bytes=16)
    rc = load().ace_bandwidth_probe(PROBE_KINDS[kind], _stream(stream), _ptr(buf),
                                    buf.numel() * buf.element_size(), int(blocks))
    if rc != 0:
        raise RuntimeError("ace_bandwidth_probe(%s) returned %d" % (kind, rc))
