"""Python binding of libmsibm (ctypes).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  torch supplies device memory and the current HIP stream; outputs are
allocated with torch.empty on the inputs' device, and calls are asynchronous on
torch's current stream like any torch op.

The library must be built (`python -m paper_1901_09593_amd.build`); importing
this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmsibm.so")

MSIBM_U8 = 0
MSIBM_F32 = 1
FLAG_BATCHED = 1
FLAG_GRAPH = 2
FLAG_PERSISTENT = 4  # switched off: calls with it fail with MsibmError
FLAG_PREBLUR = 8     # plain and batched forward: level 0 matched on the blurred input
FLAG_MEDIAN = 16     # plain and batched forward: selective median filter (Eq. 10) at every hard level
FLAG_GATED = 32      # plain and batched forward: confidence gating (Eqs. 5-9) at every hard level
MAX_LEVELS = 8


class MsibmError(RuntimeError):
    """A libmsibm call returned a negative status."""

    def __init__(self, status: int, message: str):
        super().__init__(f"msibm status {status}: {message}")
        self.status = status


class Pair(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("max_disp", ctypes.c_int32), ("num_levels", ctypes.c_int32)]


MAX_LEVELS = 8


class Config(ctypes.Structure):
    _fields_ = [("half_window", ctypes.c_int32), ("refine_radius", ctypes.c_int32),
                ("var_eps", ctypes.c_float), ("soft_radius", ctypes.c_int32),
                ("tau", ctypes.c_float), ("flags", ctypes.c_int32),
                ("half_window_levels", ctypes.c_int32 * MAX_LEVELS),
                ("median_alpha", ctypes.c_float),
                ("gate_alpha", ctypes.c_float),
                ("gate_beta", ctypes.c_float)]


_lib = None
_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_PP = ctypes.POINTER(ctypes.c_void_p)


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1901_09593_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.msibm_last_error.restype = ctypes.c_char_p
        L.msibm_version.restype = ctypes.c_char_p
        L.msibm_pyramid.argtypes = [_VP, _I32, _I32, _I32, _I32, _I32, _PP,
                                    ctypes.POINTER(_I32), _VP]
        L.msibm_pyramid.restype = _I32
        L.msibm_median_filter.argtypes = [_VP, _I32, _VP, _I32, _I32, _I32, ctypes.c_double, _VP,
                                          _I32, _VP]
        L.msibm_median_filter.restype = _I32
        L.msibm_upsample_cost.argtypes = [_VP, _I32, _I32, _I32, _I32, _I32, _VP, _I32, _VP]
        L.msibm_upsample_cost.restype = _I32
        L.msibm_match_level_gated.argtypes = [_VP, _VP, _I32, _I32, _I32, _I32, _I32, _I32, _VP, _VP,
                                              _I32, _I32, _I32, _I32, ctypes.c_double, ctypes.c_float,
                                              _VP, _VP, _I32, _VP, ctypes.c_size_t, _VP]
        L.msibm_match_level_gated.restype = _I32
        L.msibm_aggregate_refine.argtypes = [_VP, _VP, _I32, _I32, _I32, _I32, _I32, _I32, _VP, _VP,
                                             _I32, ctypes.c_double, ctypes.c_float, _VP, ctypes.c_size_t,
                                             _VP]
        L.msibm_aggregate_refine.restype = _I32
        L.msibm_pyramid_adjoint.argtypes = [_VP, _I32, _I32, _I32, _VP, _I32, _I32, _I32, _VP]
        L.msibm_pyramid_adjoint.restype = _I32
        L.msibm_levels_workspace_size.argtypes = [ctypes.POINTER(Pair), ctypes.POINTER(Config)]
        L.msibm_levels_workspace_size.restype = ctypes.c_size_t
        L.msibm_disparity_levels.argtypes = [ctypes.POINTER(Pair), ctypes.POINTER(Config), _PP, _PP, _VP,
                                             ctypes.c_size_t, _VP]
        L.msibm_disparity_levels.restype = _I32
        L.msibm_backward_levels.argtypes = [ctypes.POINTER(Pair), ctypes.POINTER(Config), _PP, _PP, _VP, _VP,
                                            _VP, ctypes.c_size_t, _VP]
        L.msibm_backward_levels.restype = _I32
        L.msibm_level_workspace_size.argtypes = [_I32, _I32]
        L.msibm_level_workspace_size.restype = ctypes.c_size_t
        L.msibm_match_level.argtypes = [_VP, _VP, _I32, _I32, _I32, _I32, _I32, _I32, _VP, _I32,
                                        _I32, _I32, _I32, ctypes.c_float, _VP, _VP, _I32, _VP, _VP,
                                        ctypes.c_size_t, _VP]
        L.msibm_match_level.restype = _I32
        L.msibm_workspace_size.argtypes = [ctypes.POINTER(Pair), _I32, ctypes.POINTER(Config)]
        L.msibm_workspace_size.restype = ctypes.c_size_t
        L.msibm_disparity.argtypes = [ctypes.POINTER(Pair), _I32, ctypes.POINTER(Config), _PP, _PP,
                                      _PP, _PP, _VP, ctypes.c_size_t, _VP]
        L.msibm_disparity.restype = _I32
        L.msibm_disparity_noalloc.argtypes = [ctypes.POINTER(Pair), ctypes.POINTER(Config), _VP, _VP, _VP, _VP,
                                              _VP]
        L.msibm_disparity_noalloc.restype = _I32
        L.msibm_backward.argtypes = [ctypes.POINTER(Pair), _I32, ctypes.POINTER(Config), _PP, _PP,
                                     _PP, _PP, _VP, ctypes.c_size_t, _VP]
        L.msibm_backward.restype = _I32
        L.msibm_fwd_bwd_l1.argtypes = [ctypes.POINTER(Pair), _I32, ctypes.POINTER(Config), _PP, _PP, _PP, _PP,
                                       _PP, _PP, _PP, _PP, _PP, _VP, ctypes.c_size_t, _VP]
        L.msibm_fwd_bwd_l1.restype = _I32
        L.msibm_force_variant.argtypes = [_I32]
        L.msibm_force_variant.restype = _I32
        L.msibm_autotune.argtypes = [_I32, ctypes.c_char_p]
        L.msibm_autotune.restype = _I32
        L.msibm_autotune_table.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        L.msibm_autotune_table.restype = ctypes.c_int64
        L.msibm_timing_enable.argtypes = [_I32]
        L.msibm_timing_enable.restype = _I32
        L.msibm_timing_read.argtypes = [_I32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_I32)]
        L.msibm_timing_read.restype = _I32
        _lib = L
    return _lib


def version() -> str:
    return lib().msibm_version().decode()


def _check(status: int):
    if status != 0:
        raise MsibmError(status, lib().msibm_last_error().decode())


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts: Sequence[Optional[torch.Tensor]]):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint8:
        return MSIBM_U8
    if t.dtype == torch.float32:
        return MSIBM_F32
    raise TypeError(f"images must be uint8 or float32, got {t.dtype}")


def _image(t: torch.Tensor) -> torch.Tensor:
    if t.dim() != 2 or not t.is_cuda:
        raise ValueError("images must be 2-D device tensors")
    if t.stride(1) != 1:
        t = t.contiguous()
    return t


def level_dim(v: int, k: int) -> int:
    for _ in range(k):
        v = (v + 1) // 2
    return v


def level_range(D: int, k: int) -> int:
    return -(-D // (1 << k))


def auto_levels(D: int) -> int:
    k = 1
    while level_range(D, k - 1) > 32 and k < MAX_LEVELS:
        k += 1
    return k


def make_config(n, r: int, var_eps: float, soft_radius: int = 0, tau: float = 0.05,
                flags: int = 0, median_alpha: Optional[float] = None,
                gate: Optional[Tuple[float, float]] = None) -> Config:
    """n: the window half-width, or a sequence of per-level half-widths (level 0
    first; levels past its end keep its last entry).  median_alpha: switch on the
    selective median filter with that threshold.  gate = (alpha, beta): switch on
    the confidence gating with those thresholds."""
    if median_alpha is not None:
        flags |= FLAG_MEDIAN
    if gate is not None:
        flags |= FLAG_GATED
    alpha = float(median_alpha) if median_alpha is not None else 0.0
    ga, gb = (float(gate[0]), float(gate[1])) if gate is not None else (0.0, 0.0)
    if isinstance(n, int):
        per = (ctypes.c_int32 * MAX_LEVELS)()
        n0 = n
    else:
        ns = [int(v) for v in n]
        if not ns or len(ns) > MAX_LEVELS:
            raise ValueError(f"1..{MAX_LEVELS} per-level half-widths")
        per = (ctypes.c_int32 * MAX_LEVELS)(*(ns + [ns[-1]] * (MAX_LEVELS - len(ns))))
        n0 = ns[0]
    return Config(n0, r, float(var_eps), soft_radius, float(tau), flags, per, alpha, ga, gb)


def force_variant(v: int = -1):
    """Pin the matching kernel shape (bit 1: right statistics staged in LDS for
    full searches, bit 2: XCD-aware tile order, bit 4: candidates split over the
    waves of 2-row tiles for full searches, bit 8: fixed candidate window for
    restricted searches); -1 = automatic."""
    _check(lib().msibm_force_variant(int(v)))


def autotune(enable: bool = True, cache_path: Optional[str] = None):
    """Measure every matching kernel shape on first use of each level shape and
    keep the fastest (optionally persisted in a text cache)."""
    _check(lib().msibm_autotune(1 if enable else 0, cache_path.encode() if cache_path else None))


def autotune_table() -> List[Tuple[int, ...]]:
    """The tuning table: (mode, n, nc, dtype, H, W, Dk, variant, microseconds)."""
    n = lib().msibm_autotune_table(None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().msibm_autotune_table(buf, len(buf))
    rows = []
    for line in buf.value.decode().splitlines():
        f = line.split()
        rows.append(tuple(int(x) for x in f[:8]) + (float(f[8]),))
    return rows


def timing_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events (clears totals)."""
    _check(lib().msibm_timing_enable(1 if on else 0))


def timing_read() -> Dict[str, Tuple[float, int]]:
    """{label: (total ms, launches)} of the timed launches so far (waits for them)."""
    cap = 256
    labels = ctypes.create_string_buffer(64 * cap)
    tot = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int32 * cap)()
    m = lib().msibm_timing_read(cap, labels, tot, cnt)
    out = {}
    for i in range(m):
        name = labels.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[name] = (tot[i], cnt[i])
    return out


# ------------------------------------------------------------------ entry points

def pyramid(img: torch.Tensor, K: int) -> List[torch.Tensor]:
    """K-level binomial pyramid of one image; level 0 is the float copy."""
    img = _image(img)
    H, W = img.shape
    levels = [torch.empty((level_dim(H, k), level_dim(W, k)), dtype=torch.float32, device=img.device)
              for k in range(K)]
    ptrs = _ptr_array(levels)
    pitches = (ctypes.c_int32 * K)(*[l.shape[1] for l in levels])
    _check(lib().msibm_pyramid(_ptr(img), _dtype_code(img), H, W, img.stride(0), K, ptrs, pitches,
                               _stream(img.device)))
    return levels


def match_level(L: torch.Tensor, R: torch.Tensor, n: int, Dk: int,
                prior: Optional[torch.Tensor] = None, r: int = 2, var_eps: float = 0.065,
                with_cost: bool = True, with_costvol: bool = False):
    """Winner-take-all of one level; prior = level k+1 map (int16) or None.
    Returns (d, C), or (d, C, V) with V the H x W x D_k scores of every scored
    candidate (-2 elsewhere) when with_costvol."""
    L = _image(L)
    R = _image(R)
    if L.shape != R.shape or L.dtype != R.dtype or L.stride(0) != R.stride(0):
        raise ValueError("left and right must share shape, dtype and pitch")
    H, W = L.shape
    dev = L.device
    d = torch.empty((H, W), dtype=torch.int16, device=dev)
    C = torch.empty((H, W), dtype=torch.float32, device=dev) if with_cost else None
    ws_bytes = lib().msibm_level_workspace_size(H, W)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if prior is not None:
        prior = prior.contiguous()
        Hc, Wc, pp = prior.shape[0], prior.shape[1], prior.stride(0)
    else:
        Hc = Wc = pp = 0
    V = torch.empty((H, W, Dk), dtype=torch.float32, device=dev) if with_costvol else None
    _check(lib().msibm_match_level(_ptr(L), _ptr(R), _dtype_code(L), H, W, L.stride(0), n, Dk,
                                   _ptr(prior), Hc, Wc, pp, r, float(var_eps), _ptr(d), _ptr(C), W,
                                   _ptr(V), _ptr(ws), ws_bytes, _stream(dev)))
    return (d, C, V) if with_costvol else (d, C)


def median_filter(d: torch.Tensor, cost: torch.Tensor, alpha: float) -> torch.Tensor:
    """Selective median filter (Eq. 10) of one int16 map given its float costs."""
    if d.dtype != torch.int16 or cost.dtype != torch.float32 or d.shape != cost.shape or d.dim() != 2:
        raise ValueError("an int16 map and a float cost map of one shape")
    if d.stride(1) != 1 or cost.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    H, W = d.shape
    out = torch.empty((H, W), dtype=torch.int16, device=d.device)
    _check(lib().msibm_median_filter(_ptr(d), d.stride(0), _ptr(cost), cost.stride(0), H, W,
                                     float(alpha), _ptr(out), W, _stream(d.device)))
    return out


def upsample_cost(coarse: torch.Tensor, H: int, W: int) -> torch.Tensor:
    """The bicubic doubling (float64, H x W) of a coarser float cost map."""
    coarse = coarse.contiguous()
    out = torch.empty((H, W), dtype=torch.float64, device=coarse.device)
    _check(lib().msibm_upsample_cost(_ptr(coarse), coarse.shape[0], coarse.shape[1], coarse.stride(0), H, W,
                                     _ptr(out), W, _stream(coarse.device)))
    return out


def match_level_gated(L: torch.Tensor, R: torch.Tensor, n: int, Dk: int, prior: torch.Tensor,
                      prior_cost: torch.Tensor, r: int, beta: float, var_eps: float):
    """Eqs. 8-9: the restricted search around the doubled prior, the full search
    where the bicubic-doubled prior cost is <= beta.  Returns (d, C)."""
    L = _image(L)
    R = _image(R)
    if L.shape != R.shape or L.dtype != R.dtype or L.stride(0) != R.stride(0):
        raise ValueError("left and right must share shape, dtype and pitch")
    prior = prior.contiguous()
    prior_cost = prior_cost.contiguous()
    if prior.shape != prior_cost.shape or prior_cost.dtype != torch.float32:
        raise ValueError("prior and prior_cost: one shape, int16 and float")
    H, W = L.shape
    dev = L.device
    d = torch.empty((H, W), dtype=torch.int16, device=dev)
    C = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws_bytes = lib().msibm_level_workspace_size(H, W)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    _check(lib().msibm_match_level_gated(_ptr(L), _ptr(R), _dtype_code(L), H, W, L.stride(0), n, Dk,
                                         _ptr(prior), _ptr(prior_cost), prior.shape[0], prior.shape[1],
                                         prior.stride(0), r, float(beta), float(var_eps), _ptr(d), _ptr(C), W,
                                         _ptr(ws), ws_bytes, _stream(dev)))
    return d, C


def aggregate_refine(L: torch.Tensor, R: torch.Tensor, n: int, Dk: int, d: torch.Tensor, C: torch.Tensor,
                     alpha: float, var_eps: float):
    """Eqs. 5-7 on copies of (d, C): pixels with C <= alpha re-picked by the
    5x5-averaged scores.  Returns the new (d, C)."""
    L = _image(L)
    R = _image(R)
    if L.shape != R.shape or L.dtype != R.dtype or L.stride(0) != R.stride(0):
        raise ValueError("left and right must share shape, dtype and pitch")
    H, W = L.shape
    dev = L.device
    d = d.to(torch.int16).contiguous().clone()
    C = C.to(torch.float32).contiguous().clone()
    if d.shape != (H, W) or C.shape != (H, W):
        raise ValueError("map and cost must have the image's shape")
    ws_bytes = lib().msibm_level_workspace_size(H, W)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    _check(lib().msibm_aggregate_refine(_ptr(L), _ptr(R), _dtype_code(L), H, W, L.stride(0), n, Dk, _ptr(d),
                                        _ptr(C), W, float(alpha), float(var_eps), _ptr(ws), ws_bytes,
                                        _stream(dev)))
    return d, C


def _pairs(lefts, rights, Ds, Ks) -> Tuple[ctypes.Array, list]:
    n = len(lefts)
    arr = (Pair * n)()
    keep = []
    for i in range(n):
        L = _image(lefts[i])
        R = _image(rights[i])
        if L.shape != R.shape or L.dtype != R.dtype or L.stride(0) != R.stride(0):
            raise ValueError("left and right must share shape, dtype and pitch")
        keep += [L, R]
        arr[i] = Pair(L.data_ptr(), R.data_ptr(), _dtype_code(L), L.shape[0], L.shape[1],
                      L.stride(0), int(Ds[i]), int(Ks[i]))
    return arr, keep


def workspace_bytes(pairs_arr, n: int, cfg: Config) -> int:
    b = lib().msibm_workspace_size(pairs_arr, n, ctypes.byref(cfg))
    if b == 0:
        raise MsibmError(-1, "invalid pairs or config: " + lib().msibm_last_error().decode())
    return b


def disparity(L: torch.Tensor, R: torch.Tensor, D: int, K: int, n: int, r: int, var_eps: float,
              soft_radius: int = 0, tau: float = 0.05, with_cost: bool = True,
              with_prior1: bool = False, preblur: bool = False,
              median_alpha: Optional[float] = None,
              gate: Optional[Tuple[float, float]] = None) -> Dict[str, torch.Tensor]:
    """Hierarchical forward pass of one pair.  Returns a dict with 'disp'
    (int16), 'cost' (float, optional), 'soft' (float, if soft_radius > 0) and
    'prior1' (int16 level-1 map, if requested or soft).  preblur: match level 0
    on the input blurred with the pyramid's kernel.  median_alpha: run the
    selective median filter with that threshold after every hard level.
    gate = (alpha, beta): the confidence gating of Eqs. 5-9 at every hard level."""
    out = disparity_many([L], [R], [D], [K], n, r, var_eps, soft_radius, tau, with_cost,
                         with_prior1, flags=FLAG_PREBLUR if preblur else 0,
                         median_alpha=median_alpha, gate=gate)
    return out[0]


def disparity_many(lefts: Sequence[torch.Tensor], rights: Sequence[torch.Tensor], Ds: Sequence[int],
                   Ks: Sequence[int], n: int, r: int, var_eps: float, soft_radius: int = 0,
                   tau: float = 0.05, with_cost: bool = True, with_prior1: bool = False,
                   flags: int = 0, workspace: Optional[torch.Tensor] = None,
                   outputs: Optional[List[Dict[str, torch.Tensor]]] = None,
                   median_alpha: Optional[float] = None,
                   gate: Optional[Tuple[float, float]] = None) -> List[Dict[str, torch.Tensor]]:
    """Forward pass of several pairs in one call (flags: FLAG_BATCHED, FLAG_GRAPH,
    FLAG_PREBLUR; a median_alpha or a gate, on either path).
    `workspace` and `outputs` may be passed in to reuse buffers across calls."""
    pairs, keep = _pairs(lefts, rights, Ds, Ks)
    npair = len(lefts)
    cfg = make_config(n, r, var_eps, soft_radius, tau, flags, median_alpha, gate)
    ws_bytes = workspace_bytes(pairs, npair, cfg)
    dev = lefts[0].device
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if outputs is None:
        outputs = []
        for i in range(npair):
            H, W = lefts[i].shape
            K = Ks[i] or auto_levels(Ds[i])
            o = {"disp": torch.empty((H, W), dtype=torch.int16, device=dev)}
            if with_cost:
                o["cost"] = torch.empty((H, W), dtype=torch.float32, device=dev)
            if soft_radius > 0:
                o["soft"] = torch.empty((H, W), dtype=torch.float32, device=dev)
            if (with_prior1 or soft_radius > 0) and K >= 2:
                o["prior1"] = torch.empty((level_dim(H, 1), level_dim(W, 1)), dtype=torch.int16,
                                          device=dev)
            outputs.append(o)
    disp = _ptr_array([o["disp"] for o in outputs])
    cost = _ptr_array([o.get("cost") for o in outputs]) if with_cost else None
    soft = _ptr_array([o.get("soft") for o in outputs]) if soft_radius > 0 else None
    pri = _ptr_array([o.get("prior1") for o in outputs])
    _check(lib().msibm_disparity(pairs, npair, ctypes.byref(cfg), disp, cost, soft, pri,
                                 _ptr(workspace), workspace.numel(), _stream(dev)))
    del keep
    return outputs


def disparity_noalloc(L: torch.Tensor, R: torch.Tensor, D: int, K: int, n, r: int, var_eps: float,
                      outputs: Dict[str, torch.Tensor], soft_radius: int = 0, tau: float = 0.05,
                      flags: int = 0, median_alpha: Optional[float] = None,
                      gate: Optional[Tuple[float, float]] = None) -> Dict[str, torch.Tensor]:
    """The forward of one pair through msibm_disparity_noalloc: no workspace,
    the library's own device scratch.  `outputs` holds 'disp' and optionally
    'cost', 'soft' and 'prior1' tensors, which are filled in place."""
    pairs, keep = _pairs([L], [R], [D], [K])
    cfg = make_config(n, r, var_eps, soft_radius, tau, flags, median_alpha, gate)
    _check(lib().msibm_disparity_noalloc(pairs, ctypes.byref(cfg), _ptr(outputs["disp"]),
                                         _ptr(outputs.get("cost")), _ptr(outputs.get("soft")),
                                         _ptr(outputs.get("prior1")), _stream(L.device)))
    del keep
    return outputs


def backward(L: torch.Tensor, R: torch.Tensor, prior1: torch.Tensor, grad_soft: torch.Tensor,
             D: int, K: int, n: int, r: int, var_eps: float, soft_radius: int,
             tau: float) -> Tuple[torch.Tensor, torch.Tensor]:
    """(dLoss/dL, dLoss/dR) given dLoss/d(d_soft), the level-1 prior held fixed."""
    (gL, gR), = backward_many([L], [R], [prior1], [grad_soft], [D], [K], n, r, var_eps,
                              soft_radius, tau)
    return gL, gR


def backward_many(lefts: Sequence[torch.Tensor], rights: Sequence[torch.Tensor],
                  priors: Sequence[torch.Tensor], grads: Sequence[torch.Tensor], Ds: Sequence[int],
                  Ks: Sequence[int], n: int, r: int, var_eps: float, soft_radius: int, tau: float,
                  flags: int = 0, workspace: Optional[torch.Tensor] = None,
                  outputs: Optional[List[Tuple[torch.Tensor, torch.Tensor]]] = None
                  ) -> List[Tuple[torch.Tensor, torch.Tensor]]:
    """Backward of several pairs in one call (flags: FLAG_BATCHED, FLAG_GRAPH).
    `workspace` and `outputs` may be passed in to reuse buffers across calls."""
    pairs, keep = _pairs(lefts, rights, Ds, Ks)
    npair = len(lefts)
    cfg = make_config(n, r, var_eps, soft_radius, tau, flags)
    ws_bytes = workspace_bytes(pairs, npair, cfg)
    dev = lefts[0].device
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    g = [x.contiguous().to(torch.float32) for x in grads]
    p1 = [x.contiguous() for x in priors]
    if outputs is None:
        outputs = [(torch.empty(L.shape, dtype=torch.float32, device=dev),
                    torch.empty(L.shape, dtype=torch.float32, device=dev)) for L in lefts]
    _check(lib().msibm_backward(pairs, npair, ctypes.byref(cfg), _ptr_array(p1), _ptr_array(g),
                                _ptr_array([o[0] for o in outputs]),
                                _ptr_array([o[1] for o in outputs]), _ptr(workspace),
                                workspace.numel(), _stream(dev)))
    del keep, g, p1
    return outputs


def fwd_bwd_l1(lefts: Sequence[torch.Tensor], rights: Sequence[torch.Tensor], gts: Sequence[torch.Tensor],
               masks: Sequence[torch.Tensor], Ds: Sequence[int], Ks: Sequence[int], n: int, r: int,
               var_eps: float, soft_radius: int, tau: float, flags: int = 0, with_cost: bool = False,
               workspace: Optional[torch.Tensor] = None,
               outputs: Optional[List[Dict[str, torch.Tensor]]] = None) -> List[Dict[str, torch.Tensor]]:
    """Forward, masked mean-L1 loss (targets `gts`, uint8 `masks`) and backward
    of several float pairs in one msibm_fwd_bwd_l1 call.  Returns per pair a
    dict with 'disp', 'soft', 'prior1', 'grad_left', 'grad_right', 'loss' (a
    one-element float tensor) and optionally 'cost'."""
    pairs, keep = _pairs(lefts, rights, Ds, Ks)
    npair = len(lefts)
    cfg = make_config(n, r, var_eps, soft_radius, tau, flags)
    ws_bytes = workspace_bytes(pairs, npair, cfg)
    dev = lefts[0].device
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    if outputs is None:
        outputs = []
        for i in range(npair):
            H, W = lefts[i].shape
            o = {"disp": torch.empty((H, W), dtype=torch.int16, device=dev),
                 "soft": torch.empty((H, W), dtype=torch.float32, device=dev),
                 "prior1": torch.empty((level_dim(H, 1), level_dim(W, 1)), dtype=torch.int16, device=dev),
                 "grad_left": torch.empty((H, W), dtype=torch.float32, device=dev),
                 "grad_right": torch.empty((H, W), dtype=torch.float32, device=dev),
                 "loss": torch.empty(1, dtype=torch.float32, device=dev)}
            if with_cost:
                o["cost"] = torch.empty((H, W), dtype=torch.float32, device=dev)
            outputs.append(o)
    gt = [g.contiguous() for g in gts]
    mk = [m.to(torch.uint8).contiguous() for m in masks]
    arrs = [_ptr_array(gt), _ptr_array(mk)] + [_ptr_array([o.get(k) for o in outputs]) for k in
                                                ("disp", "cost", "soft", "prior1", "grad_left", "grad_right",
                                                 "loss")]
    _check(lib().msibm_fwd_bwd_l1(pairs, npair, ctypes.byref(cfg), *arrs, _ptr(workspace), workspace.numel(),
                                  _stream(dev)))
    del keep
    return outputs


class MsibmFunction(torch.autograd.Function):
    """d_soft = MsibmFunction.apply(L, R, D, K, n, r, var_eps, soft_radius, tau).

    Forward runs the whole hierarchy (soft-argmax at level 0); backward returns
    dLoss/dL and dLoss/dR through the level-0 scores with the level-1 prior held
    fixed.  L and R are float32 device images."""

    @staticmethod
    def forward(ctx, L, R, D, K, n, r, var_eps, soft_radius, tau):
        out = disparity(L, R, D, K, n, r, var_eps, soft_radius, tau, with_cost=False,
                        with_prior1=True)
        ctx.save_for_backward(L, R, out["prior1"])
        ctx.params = (D, K, n, r, var_eps, soft_radius, tau)
        ctx.mark_non_differentiable(out["disp"])
        return out["soft"], out["disp"]

    @staticmethod
    def backward(ctx, grad_soft, grad_disp):
        L, R, p1 = ctx.saved_tensors
        D, K, n, r, var_eps, soft_radius, tau = ctx.params
        if grad_soft is None:
            grad_soft = torch.zeros_like(L)
        gL, gR = backward(L, R, p1, grad_soft, D, K, n, r, var_eps, soft_radius, tau)
        return gL, gR, None, None, None, None, None, None, None


# ------------------------------------------------ soft output at every level

def pyramid_adjoint(g_coarse: torch.Tensor, H: int, W: int,
                    g_fine: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g_fine + reduce^T(g_coarse) (g_fine = zeros when not given)."""
    g_coarse = g_coarse.contiguous()
    if g_fine is None:
        g_fine = torch.zeros((H, W), dtype=torch.float32, device=g_coarse.device)
    _check(lib().msibm_pyramid_adjoint(_ptr(g_coarse), g_coarse.shape[0], g_coarse.shape[1], g_coarse.stride(0),
                                       _ptr(g_fine), H, W, g_fine.stride(0), _stream(g_coarse.device)))
    return g_fine


def _levels_setup(L, R, D, K, n, var_eps, soft_radius, tau):
    pairs, keep = _pairs([L], [R], [D], [K])
    cfg = make_config(n, 0, var_eps, soft_radius, tau)
    b = lib().msibm_levels_workspace_size(pairs, ctypes.byref(cfg))
    if b == 0:
        raise MsibmError(-1, "invalid pair or config: " + lib().msibm_last_error().decode())
    ws = torch.empty(b, dtype=torch.uint8, device=L.device)
    Kr = K or auto_levels(D)
    shapes = [(level_dim(L.shape[0], k), level_dim(L.shape[1], k)) for k in range(Kr)]
    return pairs, keep, cfg, ws, Kr, shapes


def disparity_levels(L: torch.Tensor, R: torch.Tensor, D: int, K: int, n, var_eps: float, soft_radius: int,
                     tau: float):
    """Soft output at every level below the coarsest.  Returns (soft, maps):
    soft[k] (float, k < K-1) and maps[k] (int16, every level)."""
    pairs, keep, cfg, ws, K, shapes = _levels_setup(L, R, D, K, n, var_eps, soft_radius, tau)
    dev = L.device
    soft = [torch.empty(sh, dtype=torch.float32, device=dev) for sh in shapes[:-1]]
    maps = [torch.empty(sh, dtype=torch.int16, device=dev) for sh in shapes]
    _check(lib().msibm_disparity_levels(pairs, ctypes.byref(cfg), _ptr_array(soft + [None]), _ptr_array(maps),
                                        _ptr(ws), ws.numel(), _stream(dev)))
    del keep
    return soft, maps


def backward_levels(L: torch.Tensor, R: torch.Tensor, maps: Sequence[torch.Tensor],
                    grad_soft: Sequence[Optional[torch.Tensor]], D: int, K: int, n, var_eps: float,
                    soft_radius: int, tau: float) -> Tuple[torch.Tensor, torch.Tensor]:
    """(dLoss/dL, dLoss/dR) for Loss = sum_k sum grad_soft[k] d_soft^k, the maps fixed."""
    pairs, keep, cfg, ws, K, shapes = _levels_setup(L, R, D, K, n, var_eps, soft_radius, tau)
    dev = L.device
    gs = [g.contiguous() if g is not None else None for g in grad_soft]
    gL = torch.empty(shapes[0], dtype=torch.float32, device=dev)
    gR = torch.empty(shapes[0], dtype=torch.float32, device=dev)
    _check(lib().msibm_backward_levels(pairs, ctypes.byref(cfg), _ptr_array(list(maps)), _ptr_array(gs + [None]),
                                       _ptr(gL), _ptr(gR), _ptr(ws), ws.numel(), _stream(dev)))
    del keep
    return gL, gR


class MsibmLevelsFunction(torch.autograd.Function):
    """softs = MsibmLevelsFunction.apply(L, R, D, K, n, var_eps, soft_radius, tau).

    Forward: the soft output of every level below the coarsest (a tuple, level 0
    first).  Backward: dLoss/dL and dLoss/dR through every level's scores and the
    pyramid, each level's prior (the next coarser hard map) held fixed."""

    @staticmethod
    def forward(ctx, L, R, D, K, n, var_eps, soft_radius, tau):
        soft, maps = disparity_levels(L, R, D, K, n, var_eps, soft_radius, tau)
        ctx.save_for_backward(L, R, *maps)
        ctx.params = (D, K, n, var_eps, soft_radius, tau)
        return tuple(soft)

    @staticmethod
    def backward(ctx, *grad_soft):
        L, R, *maps = ctx.saved_tensors
        D, K, n, var_eps, soft_radius, tau = ctx.params
        gL, gR = backward_levels(L, R, maps, list(grad_soft), D, K, n, var_eps, soft_radius, tau)
        return gL, gR, None, None, None, None, None, None
