"""Thin Python binding of the wsgrid C-ABI (include/wsgrid.h).

Argument marshalling only: every step of gridding and degridding runs in the
HIP library ``libwsgrid.so``.  PyTorch supplies device memory and the stream.
The functions carry the C names; ``Plan`` wraps them for tensors.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsgrid.so")
HEADER = os.path.join(HERE, "..", "include", "wsgrid.h")

WSG_F32, WSG_F64 = 0, 1
WSG_IMPROVED, WSG_IMPROVED_NO_OFFSET, WSG_ORIGINAL = 0, 1, 2
METHODS = {"improved": WSG_IMPROVED, "no_offset": WSG_IMPROVED_NO_OFFSET, "original": WSG_ORIGINAL}
WSG_OK, WSG_EINVAL, WSG_EWORKSPACE, WSG_ENOMEM, WSG_EHIP = 0, -1, -2, -3, -4

_lib = None
_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)

_SIGNATURES = {
    "grid_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "grid_create_variant": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int]),
    "grid_create_axes": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int]),
    "grid_plan_axes": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, _c_double_p, _c_int_p, _c_double_p, _c_int_p,
                                      _c_int_p, _c_double_p]),
    "wsg_plan_params_axes": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, _c_int_p, _c_int_p, _c_int_p, _c_double_p,
                                            _c_double_p]),
    "grid_destroy": (None, [ctypes.c_void_p]),
    "grid_plan_info": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, _c_int_p, _c_int_p, _c_double_p, _c_double_p,
                                      _c_double_p]),
    "grid_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]),
    "grid_workspace_bytes_min": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]),
    "grid_visibilities": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]),
    "degrid_visibilities": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "grid_visibilities_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int64_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_size_t, ctypes.c_void_p]),
    "degrid_visibilities_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int64_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]),
    "grid_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int64_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "grid_visibilities_prepared": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "degrid_visibilities_prepared": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                                    ctypes.c_void_p]),
    "grid_workspace_bytes_batch": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                                     ctypes.c_int]),
    "grid_visibilities_multi": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _c_int64_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_size_t, ctypes.c_void_p]),
    "degrid_visibilities_multi": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _c_int64_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]),
    "grid_workspace_bytes_multi": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _c_int64_p,
                                                     ctypes.c_int]),
    "grid_layers_per_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                            ctypes.c_size_t]),
    "grid_skipped": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "grid_last_skipped": (ctypes.c_int64, [ctypes.c_void_p]),
    "grid_visibilities_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "wsg_bandwidth_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "grid_last_error": (ctypes.c_char_p, []),
    "wsg_design_eval": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, _c_double_p, _c_double_p,
                                       ctypes.c_int, _c_double_p, _c_double_p, _c_double_p]),
    "wsg_stage_timing": (None, [ctypes.c_int]),
    "wsg_stage_times": (ctypes.c_int, [_c_double_p, _c_int_p, ctypes.c_int]),
    "wsg_plan_params": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, _c_int_p, _c_int_p, _c_int_p, _c_double_p,
                                       _c_double_p]),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/wsgrid.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"defined"})


def lib() -> ctypes.CDLL:
    """Load libwsgrid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2101_11172_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _err(rc: int, what: str):
    if rc != WSG_OK:
        raise RuntimeError(f"{what} failed ({rc}): {lib().grid_last_error().decode()}")


# ---- the C entry points, by name -------------------------------------------

def grid_create(N: int, L: float, W: int, x0: float, wmax: float) -> int:
    p = lib().grid_create(N, L, W, x0, wmax)
    if not p:
        raise RuntimeError(f"grid_create failed: {lib().grid_last_error().decode()}")
    return p


def grid_create_variant(N: int, L: float, W: int, x0: float, wmax: float, z_offset: bool) -> int:
    p = lib().grid_create_variant(N, L, W, x0, wmax, 1 if z_offset else 0)
    if not p:
        raise RuntimeError(f"grid_create_variant failed: {lib().grid_last_error().decode()}")
    return p


def grid_create_axes(N: int, L: float, W: int, x0: float, Wz: int, z0: float, wmax: float, method: int,
                     n_bins: int = 0) -> int:
    p = lib().grid_create_axes(N, L, W, x0, Wz, z0, wmax, method, n_bins)
    if not p:
        raise RuntimeError(f"grid_create_axes failed: {lib().grid_last_error().decode()}")
    return p


def grid_plan_axes(plan: int) -> dict:
    W, Wz, method, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    x0, z0, Ez = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _err(lib().grid_plan_axes(plan, W, x0, Wz, z0, method, nb, Ez), "grid_plan_axes")
    return dict(W=W.value, x0=x0.value, Wz=Wz.value, z0=z0.value, method=method.value, n_bins=nb.value,
                E_z=Ez.value)


def wsg_plan_params_axes(N: int, L: float, W: int, x0: float, Wz: int, z0: float, wmax: float, method: int,
                         n_bins: int = 0) -> dict:
    Np, tlo, thi = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    n0, ns = ctypes.c_double(), ctypes.c_double()
    _err(lib().wsg_plan_params_axes(N, L, W, x0, Wz, z0, wmax, method, n_bins, Np, tlo, thi, n0, ns),
         "wsg_plan_params_axes")
    return dict(Nprime=Np.value, t_lo=tlo.value, t_hi=thi.value, n0=n0.value, n_scale=ns.value)


def grid_destroy(plan: int) -> None:
    lib().grid_destroy(plan)


def grid_plan_info(plan: int) -> dict:
    Np, tlo, nl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    n0, ns, E = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _err(lib().grid_plan_info(plan, Np, nl, tlo, n0, ns, E), "grid_plan_info")
    return dict(Nprime=Np.value, t_lo=tlo.value, n_layers=nl.value, n0=n0.value, n_scale=ns.value, E=E.value)


def grid_workspace_bytes(plan: int, prec: int, M: int) -> int:
    n = lib().grid_workspace_bytes(plan, prec, M)
    if n == 0:
        raise RuntimeError("grid_workspace_bytes: bad argument")
    return n


def grid_workspace_bytes_min(plan: int, prec: int, M: int) -> int:
    n = lib().grid_workspace_bytes_min(plan, prec, M)
    if n == 0:
        raise RuntimeError("grid_workspace_bytes_min: bad argument")
    return n


def grid_visibilities(plan: int, prec: int, M: int, uvw_ptr: int, vis_ptr: int, dirty_ptr: int,
                      ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _err(lib().grid_visibilities(plan, prec, M, uvw_ptr, vis_ptr, dirty_ptr, ws_ptr, ws_bytes, stream),
         "grid_visibilities")


def grid_visibilities_noalloc(plan: int, prec: int, M: int, uvw_ptr: int, vis_ptr: int, dirty_ptr: int,
                              stream: int) -> None:
    _err(lib().grid_visibilities_noalloc(plan, prec, M, uvw_ptr, vis_ptr, dirty_ptr, stream),
         "grid_visibilities_noalloc")


def degrid_visibilities(plan: int, prec: int, M: int, uvw_ptr: int, image_ptr: int, vis_ptr: int,
                        ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _err(lib().degrid_visibilities(plan, prec, M, uvw_ptr, image_ptr, vis_ptr, ws_ptr, ws_bytes, stream),
         "degrid_visibilities")


def _counts(M) -> ctypes.Array:
    return (ctypes.c_int64 * len(M))(*[int(m) for m in M])


def grid_workspace_bytes_batch(plan: int, prec: int, nch: int, M: int, min_passes: bool = False) -> int:
    n = lib().grid_workspace_bytes_batch(plan, prec, nch, M, 1 if min_passes else 0)
    if n == 0:
        raise RuntimeError("grid_workspace_bytes_batch: bad argument")
    return n


def grid_layers_per_pass(plan: int, prec: int, nch: int, M: int, ws_bytes: int) -> int:
    n = lib().grid_layers_per_pass(plan, prec, nch, M, ws_bytes)
    if n <= 0:
        raise RuntimeError(f"grid_layers_per_pass failed: {grid_last_error()}")
    return n


def grid_visibilities_batch(plan: int, prec: int, M, uvw_ptr: int, vis_ptr: int, dirty_ptr: int,
                            ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _err(lib().grid_visibilities_batch(plan, prec, len(M), _counts(M), uvw_ptr, vis_ptr, dirty_ptr, ws_ptr,
                                       ws_bytes, stream), "grid_visibilities_batch")


def degrid_visibilities_batch(plan: int, prec: int, M, uvw_ptr: int, image_ptr: int, vis_ptr: int,
                              ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _err(lib().degrid_visibilities_batch(plan, prec, len(M), _counts(M), uvw_ptr, image_ptr, vis_ptr, ws_ptr,
                                         ws_bytes, stream), "degrid_visibilities_batch")


def grid_prepare(plan: int, prec: int, M, uvw_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _err(lib().grid_prepare(plan, prec, len(M), _counts(M), uvw_ptr, ws_ptr, ws_bytes, stream), "grid_prepare")


def grid_visibilities_prepared(plan: int, prec: int, vis_ptr: int, dirty_ptr: int, ws_ptr: int, ws_bytes: int,
                               stream: int) -> None:
    _err(lib().grid_visibilities_prepared(plan, prec, vis_ptr, dirty_ptr, ws_ptr, ws_bytes, stream),
         "grid_visibilities_prepared")


def degrid_visibilities_prepared(plan: int, prec: int, image_ptr: int, vis_ptr: int, ws_ptr: int, ws_bytes: int,
                                 stream: int) -> None:
    _err(lib().degrid_visibilities_prepared(plan, prec, image_ptr, vis_ptr, ws_ptr, ws_bytes, stream),
         "degrid_visibilities_prepared")


def _plan_array(plans) -> ctypes.Array:
    return (ctypes.c_void_p * len(plans))(*[int(p) for p in plans])


def grid_visibilities_multi(plans, prec: int, M, uvw_ptr: int, vis_ptr: int, dirty_ptr: int, ws_ptr: int,
                            ws_bytes: int, stream: int) -> None:
    _err(lib().grid_visibilities_multi(len(M), _plan_array(plans), prec, _counts(M), uvw_ptr, vis_ptr, dirty_ptr,
                                       ws_ptr, ws_bytes, stream), "grid_visibilities_multi")


def degrid_visibilities_multi(plans, prec: int, M, uvw_ptr: int, image_ptr: int, vis_ptr: int, ws_ptr: int,
                              ws_bytes: int, stream: int) -> None:
    _err(lib().degrid_visibilities_multi(len(M), _plan_array(plans), prec, _counts(M), uvw_ptr, image_ptr, vis_ptr,
                                         ws_ptr, ws_bytes, stream), "degrid_visibilities_multi")


def grid_workspace_bytes_multi(plans, prec: int, M, min_passes: bool = False) -> int:
    n = lib().grid_workspace_bytes_multi(len(M), _plan_array(plans), prec, _counts(M), 1 if min_passes else 0)
    if n == 0:
        raise RuntimeError(f"grid_workspace_bytes_multi: bad argument ({grid_last_error()})")
    return n


def grid_skipped(plan: int, ws_ptr: int, stream: int) -> int:
    n = lib().grid_skipped(plan, ws_ptr, stream)
    if n < 0:
        raise RuntimeError(f"grid_skipped failed: {lib().grid_last_error().decode()}")
    return int(n)


def grid_last_skipped(plan: int) -> int:
    n = lib().grid_last_skipped(plan)
    if n < 0:
        raise RuntimeError(f"grid_last_skipped failed: {lib().grid_last_error().decode()}")
    return int(n)


def wsg_bandwidth_probe(src_ptr: int, dst_ptr: int, nbytes: int, stream: int) -> None:
    _err(lib().wsg_bandwidth_probe(src_ptr, dst_ptr, nbytes, stream), "wsg_bandwidth_probe")


def grid_last_error() -> str:
    return lib().grid_last_error().decode()


def wsg_design_eval(W: int, x0: float, nu, x):
    """Library's own design (host only): c [len(nu), W] from the device polynomials, h(x), E."""
    import numpy as np
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    c = np.zeros((nu.size, W))
    h = np.zeros(x.size)
    E = ctypes.c_double()
    dp = lambda a: a.ctypes.data_as(_c_double_p)
    _err(lib().wsg_design_eval(W, x0, nu.size, dp(nu), dp(c), x.size, dp(x), dp(h), E), "wsg_design_eval")
    return c, h, E.value


def wsg_plan_params(N: int, L: float, W: int, x0: float, wmax: float, z_offset: bool = True) -> dict:
    Np, tlo, thi = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    n0, ns = ctypes.c_double(), ctypes.c_double()
    _err(lib().wsg_plan_params(N, L, W, x0, wmax, 1 if z_offset else 0, Np, tlo, thi, n0, ns), "wsg_plan_params")
    return dict(Nprime=Np.value, t_lo=tlo.value, t_hi=thi.value, n0=n0.value, n_scale=ns.value)


STAGES = ("grid_bin", "grid_tiles", "grid_fft_v", "grid_fft_u", "degrid_bin", "degrid_fft_p", "degrid_fft_q",
          "degrid_tiles", "grid_transpose", "degrid_transpose")


def wsg_stage_timing(enable: bool) -> None:
    lib().wsg_stage_timing(1 if enable else 0)


def wsg_stage_times() -> dict:
    """{stage name: (total ms, launches)} since the last call; waits for the events."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    rc = lib().wsg_stage_times(ms, cnt, n)
    if rc < 0:
        raise RuntimeError(f"wsg_stage_times failed: {grid_last_error()}")
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}


# ---- tensor convenience ------------------------------------------------------

_PREC = {torch.complex64: WSG_F32, torch.complex128: WSG_F64, torch.float32: WSG_F32, torch.float64: WSG_F64}


class Plan:
    """Improved W-stacking plan on one HIP device (see include/wsgrid.h).

    max_workspace_bytes caps the workspace each precision allocates: below
    grid_workspace_bytes the library takes the w-layers in passes (at least
    grid_workspace_bytes_min is allocated).  z_offset=False selects the
    variant without z offset; Wz, z0 a w-axis gridding function of its own and
    method "improved" | "no_offset" | "original" (with n_bins, 0 for eq. N_w)
    select grid_create_axes.
    """

    def __init__(self, N: int, L: float, W: int, x0: float, wmax: float, device=None,
                 max_workspace_bytes: int | None = None, z_offset: bool = True, Wz: int | None = None,
                 z0: float | None = None, method: str | None = None, n_bins: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("wsgrid needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        if method is None:
            method = "improved" if z_offset else "no_offset"
        Wz = (1 if method == "original" else W) if Wz is None else Wz
        z0 = x0 if z0 is None else z0
        with torch.cuda.device(self.device):
            self._p = grid_create_axes(N, L, W, x0, Wz, z0, wmax, METHODS[method], n_bins)
        self.N, self.L, self.W, self.x0, self.wmax = N, L, W, x0, wmax
        self.axes = grid_plan_axes(self._p)
        self.max_workspace_bytes = max_workspace_bytes
        self.info = grid_plan_info(self._p)
        self._ws = {}
        self._prep = {}        # prec -> (M, channels, workspace) of the binning kept by prepare()

    def close(self):
        if getattr(self, "_p", None):
            grid_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, prec: int, M: int, nch: int = 1) -> torch.Tensor:
        """The workspace of a plain or prepare() call in this precision (such a
        call replaces the binning a previous prepare() left there)."""
        self._prep.pop(prec, None)
        need = grid_workspace_bytes_batch(self._p, prec, nch, M)
        if self.max_workspace_bytes is not None and need > self.max_workspace_bytes:
            need = max(grid_workspace_bytes_batch(self._p, prec, nch, M, True), int(self.max_workspace_bytes))
        ws = self._ws.get(prec)
        over_cap = (ws is not None and self.max_workspace_bytes is not None
                    and ws.numel() > max(need, int(self.max_workspace_bytes)))
        if ws is None or ws.numel() < need or over_cap:
            self._ws.pop(prec, None)
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[prec] = ws
        return ws

    def _check_uvw(self, uvw: torch.Tensor) -> int:
        if uvw.dtype != torch.float64 or uvw.device != self.device or uvw.dim() != 2 or uvw.shape[1] != 3 \
                or not uvw.is_contiguous():
            raise ValueError("uvw must be a contiguous float64 [M, 3] tensor on the plan's device")
        return uvw.shape[0]

    def check_batch(self, uvw: torch.Tensor, counts, vis: torch.Tensor | None = None,
                    image: torch.Tensor | None = None):
        """Validate the inputs of a batched call (raises ValueError); returns (M, counts)."""
        M = self._check_uvw(uvw)
        counts = [int(c) for c in counts]
        if not counts or min(counts) < 0 or sum(counts) != M:
            raise ValueError("counts must be non-negative and add up to the number of visibilities")
        if vis is not None and (vis.dtype not in (torch.complex64, torch.complex128) or vis.shape != (M,)
                                or not vis.is_contiguous() or vis.device != self.device):
            raise ValueError("vis must be a contiguous complex64/complex128 [M] tensor on the plan's device")
        if image is not None and (image.dtype not in (torch.float32, torch.float64)
                                  or image.shape != (len(counts), self.N, self.N)
                                  or not image.is_contiguous() or image.device != self.device):
            raise ValueError("image must be a contiguous float32/float64 [channels, N, N] tensor on the device")
        return M, counts

    def grid(self, uvw: torch.Tensor, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        M = self._check_uvw(uvw)
        if vis.dtype not in (torch.complex64, torch.complex128) or vis.shape != (M,) or not vis.is_contiguous() \
                or vis.device != self.device:
            raise ValueError("vis must be a contiguous complex64/complex128 [M] tensor on the plan's device")
        prec = _PREC[vis.dtype]
        rdt = torch.float32 if prec == WSG_F32 else torch.float64
        if out is None:
            out = torch.empty((self.N, self.N), dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != (self.N, self.N) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        ws = self.workspace(prec, M)
        grid_visibilities(self._p, prec, M, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(), ws.data_ptr(),
                          ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def degrid(self, uvw: torch.Tensor, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        M = self._check_uvw(uvw)
        if image.dtype not in (torch.float32, torch.float64) or image.shape != (self.N, self.N) \
                or not image.is_contiguous() or image.device != self.device:
            raise ValueError("image must be a contiguous float32/float64 [N, N] tensor on the plan's device")
        prec = _PREC[image.dtype]
        cdt = torch.complex64 if prec == WSG_F32 else torch.complex128
        if out is None:
            out = torch.empty(M, dtype=cdt, device=self.device)
        elif out.dtype != cdt or out.shape != (M,) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        ws = self.workspace(prec, M)
        degrid_visibilities(self._p, prec, M, uvw.data_ptr(), image.data_ptr(), out.data_ptr(), ws.data_ptr(),
                            ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def grid_batch(self, uvw: torch.Tensor, counts, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Dirty maps [len(counts), N, N] of channels whose visibilities are
        consecutive runs of counts[c] rows of uvw / entries of vis."""
        M, counts = self.check_batch(uvw, counts, vis=vis)
        prec = _PREC[vis.dtype]
        rdt = torch.float32 if prec == WSG_F32 else torch.float64
        shape = (len(counts), self.N, self.N)
        if out is None:
            out = torch.empty(shape, dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != shape or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        ws = self.workspace(prec, M, len(counts))
        grid_visibilities_batch(self._p, prec, counts, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(),
                                ws.data_ptr(), ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def degrid_batch(self, uvw: torch.Tensor, counts, image: torch.Tensor,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """Model visibilities of channels c = 0.. from images [len(counts), N, N],
        concatenated in channel order."""
        M, counts = self.check_batch(uvw, counts, image=image)
        prec = _PREC[image.dtype]
        cdt = torch.complex64 if prec == WSG_F32 else torch.complex128
        if out is None:
            out = torch.empty(M, dtype=cdt, device=self.device)
        elif out.dtype != cdt or out.shape != (M,) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        ws = self.workspace(prec, M, len(counts))
        degrid_visibilities_batch(self._p, prec, counts, uvw.data_ptr(), image.data_ptr(), out.data_ptr(),
                                  ws.data_ptr(), ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out

    # ---- one binning shared by gridding and degridding (grid_prepare) ----

    def prepare(self, uvw: torch.Tensor, dtype=torch.float32, counts=None) -> None:
        """Bin uvw once for the prepared calls that follow (precision of dtype:
        float32/complex64 or float64/complex128).  counts: channel counts as for
        grid_batch (default one channel).  Any plain call of this plan in that
        precision replaces the binning."""
        M = self._check_uvw(uvw)
        counts = [M] if counts is None else self.check_batch(uvw, counts)[1]
        prec = _PREC[dtype]
        ws = self.workspace(prec, M, len(counts))
        grid_prepare(self._p, prec, counts, uvw.data_ptr(), ws.data_ptr(), ws.numel(),
                     torch.cuda.current_stream(self.device).cuda_stream)
        self._prep[prec] = (M, len(counts), ws, self._uvw_key(uvw, counts))

    @staticmethod
    def _uvw_key(uvw: torch.Tensor, counts) -> tuple:
        return (uvw.data_ptr(), uvw._version, tuple(uvw.shape), tuple(counts))

    def _prepared(self, prec: int):
        if prec not in self._prep or self._ws.get(prec) is not self._prep[prec][2]:
            raise RuntimeError("no prepared binning in this precision: call prepare(uvw) first")
        return self._prep[prec][:3]

    def prepared_for(self, dtype, uvw: torch.Tensor | None = None, counts=None) -> bool:
        """Whether a binning from prepare() is held for this precision (and, if
        given, for this uvw tensor, unmodified since)."""
        prec = _PREC[dtype]
        if prec not in self._prep or self._ws.get(prec) is not self._prep[prec][2]:
            return False
        return uvw is None or self._prep[prec][3] == self._uvw_key(uvw, [uvw.shape[0]] if counts is None else counts)

    def grid_prepared(self, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Dirty map(s) of the prepared visibilities: [N, N] (or [channels, N, N])."""
        prec = _PREC[vis.dtype] if vis.dtype in (torch.complex64, torch.complex128) else None
        if prec is None:
            raise ValueError("vis must be complex64 or complex128")
        M, nch, ws = self._prepared(prec)
        if vis.shape != (M,) or not vis.is_contiguous() or vis.device != self.device:
            raise ValueError("vis must be a contiguous [M] tensor of the prepared visibilities on the device")
        rdt = torch.float32 if prec == WSG_F32 else torch.float64
        shape = (self.N, self.N) if nch == 1 else (nch, self.N, self.N)
        if out is None:
            out = torch.empty(shape, dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != shape or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        grid_visibilities_prepared(self._p, prec, vis.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                   torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def degrid_prepared(self, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Model visibilities [M] of the prepared uvw from image(s) [N, N] (or [channels, N, N])."""
        if image.dtype not in (torch.float32, torch.float64):
            raise ValueError("image must be float32 or float64")
        prec = _PREC[image.dtype]
        M, nch, ws = self._prepared(prec)
        shape = (self.N, self.N) if nch == 1 else (nch, self.N, self.N)
        if image.shape != shape or not image.is_contiguous() or image.device != self.device:
            raise ValueError(f"image must be a contiguous {shape} tensor on the plan's device")
        cdt = torch.complex64 if prec == WSG_F32 else torch.complex128
        if out is None:
            out = torch.empty(M, dtype=cdt, device=self.device)
        elif out.dtype != cdt or out.shape != (M,) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        degrid_visibilities_prepared(self._p, prec, image.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                     torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def skipped(self, prec: int) -> int:
        ws = self._ws[prec]
        return grid_skipped(self._p, ws.data_ptr(), torch.cuda.current_stream(self.device).cuda_stream)


class PlanSet:
    """Channels with plans of their own (grid/degrid_visibilities_multi).

    plans[c] is channel c's Plan (image size, wmax and widths per plan);
    channels that share a plan must be consecutive.  Maps are packed channel
    after channel (N_c^2 elements each); maps() gives the [N_c, N_c] views.
    max_workspace_bytes caps the workspace (layer passes below the full size).
    """

    def __init__(self, plans, max_workspace_bytes: int | None = None):
        self.plans = list(plans)
        self.device = self.plans[0].device
        if any(p.device != self.device for p in self.plans):
            raise ValueError("all plans must be on one device")
        self.max_workspace_bytes = max_workspace_bytes
        self._ws = {}
        self._prep = None          # (prec, M, counts, runs, run sizes) of the binning kept by prepare()
        self._prep_ws = []         # its workspaces, one per run

    def _ptrs(self):
        return [p._p for p in self.plans]

    def map_elements(self) -> int:
        return sum(p.N * p.N for p in self.plans)

    def maps(self, packed: torch.Tensor):
        out, off = [], 0
        for p in self.plans:
            out.append(packed[off:off + p.N * p.N].view(p.N, p.N))
            off += p.N * p.N
        return out

    def workspace(self, prec: int, counts) -> torch.Tensor:
        need = grid_workspace_bytes_multi(self._ptrs(), prec, counts)
        if self.max_workspace_bytes is not None and need > self.max_workspace_bytes:
            need = max(grid_workspace_bytes_multi(self._ptrs(), prec, counts, True), int(self.max_workspace_bytes))
        ws = self._ws.get(prec)
        if ws is None or ws.numel() < need or (self.max_workspace_bytes is not None and ws.numel() > need):
            self._ws.pop(prec, None)
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[prec] = ws
        return ws

    def _runs(self):
        """(plan, first channel, end channel) of each run of channels on one plan."""
        runs = []
        for c, p in enumerate(self.plans):
            if runs and runs[-1][0] is p:
                runs[-1][2] = c + 1
            else:
                if any(r[0] is p for r in runs):
                    raise ValueError("channels sharing a plan must be consecutive")
                runs.append([p, c, c + 1])
        return [tuple(r) for r in runs]

    # ---- one binning shared by gridding and degridding (grid_prepare per run) ----

    def prepare(self, uvw: torch.Tensor, counts, dtype=torch.float32) -> None:
        """Bin the channels' visibilities once, one grid_prepare per run of
        channels on one plan, each into a workspace of its own (each within
        max_workspace_bytes when set, but at least the smallest its run accepts;
        a run's layers go in passes below its full size).  grid_prepared / degrid_prepared then take only values."""
        M, counts = self._check(uvw, counts)
        prec = _PREC[dtype]
        runs = self._runs()
        ms = [sum(counts[c0:c1]) for _, c0, c1 in runs]
        full = [grid_workspace_bytes_batch(p._p, prec, c1 - c0, m) for (p, c0, c1), m in zip(runs, ms)]
        least = [grid_workspace_bytes_batch(p._p, prec, c1 - c0, m, True) for (p, c0, c1), m in zip(runs, ms)]
        size = full
        if self.max_workspace_bytes is not None:
            # each run's workspace within the cap (at least its smallest), as the
            # shared workspace of grid() is for every run: the runs then take the
            # same layer passes as there, and the binnings together hold up to
            # one cap per run
            cap = int(self.max_workspace_bytes)
            size = [min(f, max(lo, cap)) for f, lo in zip(full, least)]
        self._prep = None
        old = self._prep_ws
        ws = [old[i] if i < len(old) and old[i].numel() == n else torch.empty(n, dtype=torch.uint8, device=self.device)
              for i, n in enumerate(size)]
        self._prep_ws = ws
        stream = torch.cuda.current_stream(self.device).cuda_stream
        v0 = 0
        for (p, c0, c1), m, w in zip(runs, ms, ws):
            grid_prepare(p._p, prec, counts[c0:c1], uvw.data_ptr() + 24 * v0, w.data_ptr(), w.numel(), stream)
            v0 += m
        self._prep = (prec, M, counts, runs, ms)

    def _prepared(self, prec: int):
        if self._prep is None or self._prep[0] != prec:
            raise RuntimeError("no prepared binning in this precision: call prepare(uvw, counts) first")
        return self._prep

    def grid_prepared(self, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Packed dirty maps of the prepared visibilities (values in channel order)."""
        if vis.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("vis must be complex64 or complex128")
        prec, M, counts, runs, ms = self._prepared(_PREC[vis.dtype])
        if vis.shape != (M,) or not vis.is_contiguous() or vis.device != self.device:
            raise ValueError("vis must be a contiguous [M] tensor of the prepared visibilities on the device")
        rdt = torch.float32 if prec == WSG_F32 else torch.float64
        if out is None:
            out = torch.empty(self.map_elements(), dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != (self.map_elements(),) or not out.is_contiguous():
            raise ValueError("out must be the packed maps")
        cs, rs = vis.element_size(), out.element_size()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        v0, m0 = 0, 0
        for (p, c0, c1), m, w in zip(runs, ms, self._prep_ws):
            grid_visibilities_prepared(p._p, prec, vis.data_ptr() + cs * v0, out.data_ptr() + rs * m0, w.data_ptr(),
                                       w.numel(), stream)
            v0 += m
            m0 += (c1 - c0) * p.N * p.N
        return out

    def degrid_prepared(self, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Model visibilities of the prepared uvw from the packed maps."""
        if image.dtype not in (torch.float32, torch.float64):
            raise ValueError("image must be float32 or float64")
        prec, M, counts, runs, ms = self._prepared(_PREC[image.dtype])
        if image.shape != (self.map_elements(),) or not image.is_contiguous() or image.device != self.device:
            raise ValueError("image must be the packed maps on the plans' device")
        cdt = torch.complex64 if prec == WSG_F32 else torch.complex128
        if out is None:
            out = torch.empty(M, dtype=cdt, device=self.device)
        elif out.dtype != cdt or out.shape != (M,) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        cs, rs = out.element_size(), image.element_size()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        v0, m0 = 0, 0
        for (p, c0, c1), m, w in zip(runs, ms, self._prep_ws):
            degrid_visibilities_prepared(p._p, prec, image.data_ptr() + rs * m0, out.data_ptr() + cs * v0,
                                         w.data_ptr(), w.numel(), stream)
            v0 += m
            m0 += (c1 - c0) * p.N * p.N
        return out

    def _check(self, uvw, counts):
        counts = [int(c) for c in counts]
        if len(counts) != len(self.plans):
            raise ValueError("one count per channel (plan)")
        M = self.plans[0]._check_uvw(uvw)
        if min(counts) < 0 or sum(counts) != M:
            raise ValueError("counts must be non-negative and add up to the number of visibilities")
        return M, counts

    def grid(self, uvw: torch.Tensor, counts, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        M, counts = self._check(uvw, counts)
        if vis.dtype not in (torch.complex64, torch.complex128) or vis.shape != (M,) or not vis.is_contiguous() \
                or vis.device != self.device:
            raise ValueError("vis must be a contiguous complex64/complex128 [M] tensor on the plans' device")
        prec = _PREC[vis.dtype]
        rdt = torch.float32 if prec == WSG_F32 else torch.float64
        if out is None:
            out = torch.empty(self.map_elements(), dtype=rdt, device=self.device)
        elif out.dtype != rdt or out.shape != (self.map_elements(),) or not out.is_contiguous():
            raise ValueError("out must be the packed maps")
        ws = self.workspace(prec, counts)
        grid_visibilities_multi(self._ptrs(), prec, counts, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(),
                                ws.data_ptr(), ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def degrid(self, uvw: torch.Tensor, counts, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        M, counts = self._check(uvw, counts)
        if image.dtype not in (torch.float32, torch.float64) or image.shape != (self.map_elements(),) \
                or not image.is_contiguous() or image.device != self.device:
            raise ValueError("image must be the packed float32/float64 maps on the plans' device")
        prec = _PREC[image.dtype]
        cdt = torch.complex64 if prec == WSG_F32 else torch.complex128
        if out is None:
            out = torch.empty(M, dtype=cdt, device=self.device)
        elif out.dtype != cdt or out.shape != (M,) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or shape")
        ws = self.workspace(prec, counts)
        degrid_visibilities_multi(self._ptrs(), prec, counts, uvw.data_ptr(), image.data_ptr(), out.data_ptr(),
                                  ws.data_ptr(), ws.numel(), torch.cuda.current_stream(self.device).cuda_stream)
        return out


class DegridFn(torch.autograd.Function):
    """Model visibilities of a real image as a differentiable torch operation.

    forward: degrid_visibilities (Algorithm 6).  backward: grid_visibilities
    (Algorithm 5) applied to the incoming gradient.  The forward bins uvw once
    (grid_prepare) and the backward reuses that binning while the plan still
    holds it for the same, unmodified uvw (else it bins again).  For a real image f and
    vis = A f, torch's gradient for a complex output is g = dL/dRe(vis) +
    i dL/dIm(vis), so dL/df = Re(A^H g); the gridding operator returns exactly
    Re(A^H g), the two being adjoint (Sec. 3.1-3.2, eq. gridded-dirty-map).
    The precision follows the image (float32 -> complex64 visibilities and a
    float32 gradient).  uvw carries no gradient.
    """

    @staticmethod
    def forward(ctx, image: torch.Tensor, plan: "Plan", uvw: torch.Tensor) -> torch.Tensor:
        ctx.plan = plan
        ctx.save_for_backward(uvw)
        image = image.contiguous()
        plan.prepare(uvw, image.dtype)
        return plan.degrid_prepared(image)

    @staticmethod
    def backward(ctx, grad_vis: torch.Tensor):
        (uvw,) = ctx.saved_tensors
        g = grad_vis.contiguous()
        if ctx.plan.prepared_for(g.dtype, uvw):
            return ctx.plan.grid_prepared(g), None, None
        return ctx.plan.grid(uvw, g), None, None


def degrid_fn(plan: Plan, uvw: torch.Tensor, image: torch.Tensor) -> torch.Tensor:
    """Differentiable degrid: DegridFn.apply(image, plan, uvw)."""
    return DegridFn.apply(image, plan, uvw)
