"""Thin Python binding of libpolymh (the C ABI in include/polymh.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch tensors carry device memory and the current HIP stream.  Names
mirror the C entry points without their ``polymh_`` prefix.  Unsigned C
arrays are exposed as signed torch tensors holding the same bits
(uint32 signatures -> int32, uint64 keys -> int64).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolymh.so")

OK, EINVAL, ERANGE, EDEVICE, ECAPACITY, ENOTSUP = 0, -1, -2, -3, -4, -5
_NAMES = {EINVAL: "EINVAL", ERANGE: "ERANGE", EDEVICE: "EDEVICE", ECAPACITY: "ECAPACITY",
          ENOTSUP: "ENOTSUP"}


class PolymhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"polymh {_NAMES.get(status, status)}: {msg}")
        self.status = status


class Box(ctypes.Structure):
    _fields_ = [("xmin", ctypes.c_int32), ("ymin", ctypes.c_int32),
                ("xmax", ctypes.c_int32), ("ymax", ctypes.c_int32)]


class Polys(ctypes.Structure):
    _fields_ = [("xy", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n", ctypes.c_int64)]


class SignConfig(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("hash_block", ctypes.c_int32), ("lds_edges", ctypes.c_int32),
                ("samples_per_lane", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

P = ctypes.c_void_p
I32, I64, U32, U64, SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
_SIGNATURES = {
    "polymh_last_error": (ctypes.c_char_p, []),
    "polymh_version": (I32, []),
    "polymh_check_device": (I32, []),
    "polymh_prepare": (I32, [P, P, P, P, P]),
    "polymh_centre": (I32, [P, P, P, P, P]),
    "polymh_box_of_workspace_size": (SZ, []),
    "polymh_box_of": (I32, [P, P, SZ, P, P]),
    "polymh_sign_default_config": (None, [P]),
    "polymh_sign_workspace_size": (SZ, [I64, P]),
    "polymh_sign": (I32, [P, Box, U64, I32, U32, P, P, P, SZ, P]),
    "polymh_sign_static": (I32, [P, Box, U64, I32, U32, P, P, P]),
    "polymh_join_rings_size": (I64, [I64, I64, I64]),
    "polymh_join_rings": (I32, [P, I64, P, I64, P, I64, P, I64, P, P, P]),
    "polymh_sign_binned_workspace_size": (SZ, [I64, I32, U32, U32, I32, P]),
    "polymh_sign_binned": (I32, [P, Box, U64, I32, U32, U32, I32, ctypes.c_double, P, P, P, SZ, P]),
    "polymh_sign_binned_prebinned": (I32, [P, Box, U64, I32, U32, U32, I32, ctypes.c_double, P, P, P, SZ, P]),
    "polymh_band": (I32, [P, I64, I32, I32, I32, U64, P, P]),
    "polymh_index_workspace_size": (SZ, [I64, I32]),
    "polymh_index_build": (I32, [P, I64, I32, P, SZ, P, P, P]),
    "polymh_query_workspace_size": (SZ, [I64, I64]),
    "polymh_query": (I32, [P, P, I64, I64, P, I64, I32, P, SZ, P, P, I64, P]),
    "polymh_refine": (I32, [P, P, P, P, I64, I64, P, P]),
    "polymh_refine_stats": (I32, [P, P, P, P, I64, I64, P, P, P]),
    "polymh_refine_workspace_size": (SZ, []),
    "polymh_refine_ws": (I32, [P, P, P, P, I64, I64, P, P, P, SZ, P]),
    "polymh_query_capped": (I32, [P, P, I64, I64, P, I64, I32, P, SZ, P, P, I64, P, P]),
    "polymh_graph_begin": (I32, [P]),
    "polymh_graph_end": (I32, [P, P]),
    "polymh_graph_launch": (I32, [P, P]),
    "polymh_graph_destroy": (None, [P]),
    "polymh_topk": (I32, [P, P, P, I64, I32, P, P, P]),
    "polymh_mlp_param_count": (I64, []),
    "polymh_mlp_bf16_count": (I64, []),
    "polymh_mlp_acts_size": (SZ, [I64]),
    "polymh_mlp_scratch_size": (SZ, [I64]),
    "polymh_mlp_sync_bf16": (I32, [P, P, P]),
    "polymh_mlp_forward": (I32, [P, I64, P, P, P, P, SZ, P]),
    "polymh_mlp_backward": (I32, [P, I64, P, P, P, SZ, P, P, P, P, SZ, P]),
    "polymh_mlp_adam": (I32, [P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, P, P]),
    "polymh_gemm_bf16": (I32, [P, I64, I64, P, I64, I64, I64, I64, I64, P, P]),
    "polymh_poly_features": (I32, [P, Box, P, P]),
    "polymh_pair_features": (I32, [P, P, P, P, I32, P, P, I64, I64, P, P]),
    "polymh_csr_rows": (I32, [P, I64, P, P]),
    "polymh_jhat": (I32, [P, P, I32, P, P, I64, P, P]),
    "polymh_rank_workspace_size": (SZ, [I64, I64, I32]),
    "polymh_rank_head": (I32, [P, P, I64, P, I32, P, P, P, P, P, P, P]),
    "polymh_scatter_scores": (I32, [P, P, I64, P, P]),
    "polymh_rank_refine": (I32, [P, P, P, P, P, I64, I64, I32, I32, ctypes.c_float, I32, P, SZ,
                                 P, P, P, P, P]),
    "polymh_rank_jhat_order": (I32, [P, P, I32, P, P, I64, P, P, P, P]),
    "polymh_rank_order": (I32, [P, I64, P, P, P, P]),
    "polymh_sig_pack_stride": (SZ, [I32]),
    "polymh_sig_pack": (I32, [P, I64, I32, P, P]),
    "polymh_rank_jhat_order_packed": (I32, [P, P, P, I32, P, P, I64, P, P, P, P]),
    "polymh_rank_head_fixed": (I32, [P, P, I64, P, I32, P, P, P, P]),
    "polymh_rank_reorder_head": (I32, [P, I64, P, P, I32, P, P, P]),
    "polymh_mlp_score_pairs": (I32, [P, P, P, P, I32, P, P, P, I64, P, P, P, P]),
    "polymh_rank_refine_ordered": (I32, [P, P, P, P, P, P, P, I64, I64, I32, I32, I32, ctypes.c_float,
                                         P, SZ, P, P, P, P]),
}


def lib():
    """Load libpolymh.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2511_16576_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != OK:
        raise PolymhError(st, lib().polymh_last_error().decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libpolymh needs a HIP device (torch.cuda.is_available() is False)")


_checked_devices = set()


def check_device():
    _require_gpu()
    d = torch.cuda.current_device()
    if d not in _checked_devices:
        _check(lib().polymh_check_device())
        _checked_devices.add(d)


@dataclasses.dataclass
class DevicePolys:
    """CSR polygons resident on the device."""
    xy: torch.Tensor        # int32 [V, 2]
    offsets: torch.Tensor   # int64 [N + 1]

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def cstruct(self) -> Polys:
        return Polys(self.xy.data_ptr(), self.offsets.data_ptr(), self.n)


def to_device(polys, device="cuda") -> DevicePolys:
    """Copy a PolySet-like object (``.xy``, ``.offsets``) to the device."""
    xy = torch.from_numpy(np.ascontiguousarray(polys.xy, dtype=np.int32).reshape(-1, 2))
    off = torch.from_numpy(np.ascontiguousarray(polys.offsets, dtype=np.int64))
    if xy.shape[0] == 0:
        xy = torch.zeros((1, 2), dtype=torch.int32)    # keep a valid pointer
    return DevicePolys(xy.to(device), off.to(device))


def _box(box) -> Box:
    if isinstance(box, Box):
        return box
    x0, y0, x1, y1 = (int(v) for v in box)
    return Box(x0, y0, x1, y1)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def default_sign_config() -> SignConfig:
    c = SignConfig()
    lib().polymh_sign_default_config(ctypes.byref(c))
    return c


def sign_config(**kw) -> SignConfig:
    c = default_sign_config()
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, int(v))
    return c


def prepare(polys: DevicePolys, stream=None):
    """(mbr int32 [N,4], area2 int64 [N], flags int32 [N])."""
    check_device()
    dev = polys.offsets.device
    n = polys.n
    mbr = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
    area2 = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    flags = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    ps = polys.cstruct()
    _check(lib().polymh_prepare(ctypes.byref(ps), _ptr(mbr), _ptr(area2), _ptr(flags), _stream(stream)))
    return mbr[:n], area2[:n], flags[:n]


def centre(polys: DevicePolys, stream=None):
    """Sec. 3.1 centring: (centred DevicePolys with the same offsets, shift
    int32 [N, 2]).  Synchronises once to check the int32 range flag."""
    check_device()
    dev = polys.offsets.device
    xy = torch.empty_like(polys.xy)
    shift = torch.empty((max(polys.n, 1), 2), dtype=torch.int32, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    ps = polys.cstruct()
    _check(lib().polymh_centre(ctypes.byref(ps), _ptr(xy), _ptr(shift), _ptr(flag), _stream(stream)))
    if int(flag.item()):
        raise ValueError("centre: a polygon spans 2^31 or more; its centred coordinates leave int32")
    return DevicePolys(xy, polys.offsets), shift[:polys.n]


@dataclasses.dataclass
class DeviceRings:
    """Polygons with holes / multipolygons resident on the device: ring r is
    xy[ring_offsets[r]:ring_offsets[r+1]], shape p owns rings
    poly_rings[p]:poly_rings[p+1]."""
    xy: torch.Tensor            # int32 [V, 2]
    ring_offsets: torch.Tensor  # int64 [R + 1]
    poly_rings: torch.Tensor    # int64 [N + 1]

    @property
    def n(self) -> int:
        return int(self.poly_rings.shape[0] - 1)


def rings_to_device(rs, device="cuda") -> DeviceRings:
    """Copy a RingSet-like object (``.xy``, ``.ring_offsets``, ``.poly_rings``)."""
    xy = torch.from_numpy(np.ascontiguousarray(rs.xy, dtype=np.int32).reshape(-1, 2))
    if xy.shape[0] == 0:
        xy = torch.zeros((1, 2), dtype=torch.int32)
    ro = torch.from_numpy(np.ascontiguousarray(rs.ring_offsets, dtype=np.int64))
    pr = torch.from_numpy(np.ascontiguousarray(rs.poly_rings, dtype=np.int64))
    return DeviceRings(xy.to(device), ro.to(device), pr.to(device))


def join_rings(R: DeviceRings, stream=None) -> DevicePolys:
    """Each shape's rings joined into one ring (``polymh_join_rings``), so
    that every other call takes shapes with holes and several components.
    Synchronises once to check the input flag."""
    check_device()
    n = R.n
    nv = int(R.xy.shape[0])
    nr = int(R.ring_offsets.shape[0] - 1)
    size = max(int(lib().polymh_join_rings_size(nv, nr, n)), 0)
    dev = R.poly_rings.device
    out = torch.empty((max(size, 1), 2), dtype=torch.int32, device=dev)
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(lib().polymh_join_rings(_ptr(R.xy), nv, _ptr(R.ring_offsets), nr, _ptr(R.poly_rings), n, _ptr(out),
                                   size, _ptr(off), _ptr(bad), _stream(stream)))
    if int(bad.item()):
        raise ValueError("join_rings: a shape without rings, or a ring with fewer than 3 vertices")
    return DevicePolys(out, off)


def box_of(polys: DevicePolys, stream=None):
    check_device()
    ws = _workspace(lib().polymh_box_of_workspace_size(), polys.offsets.device)
    out = Box()
    ps = polys.cstruct()
    _check(lib().polymh_box_of(ctypes.byref(ps), _ptr(ws), ws.numel(), ctypes.byref(out),
                               _stream(stream)))
    return (out.xmin, out.ymin, out.xmax, out.ymax)


def sign_workspace_size(n: int, config: SignConfig | None = None) -> int:
    return int(lib().polymh_sign_workspace_size(n, ctypes.byref(config) if config else None))


def sign(polys: DevicePolys, box, seed: int, k: int, cap: int, config: SignConfig | None = None,
         out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Alg. 1 signatures: int32 [N, k] holding uint32 values (0 = no hit)."""
    check_device()
    dev = polys.offsets.device
    n = polys.n
    if out is None:
        out = torch.empty((max(n, 1), k), dtype=torch.int32, device=dev)
    need = sign_workspace_size(n, config)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    ps = polys.cstruct()
    _check(lib().polymh_sign(ctypes.byref(ps), _box(box), seed & ((1 << 64) - 1), k, cap, _ptr(out),
                             ctypes.byref(config) if config else None, _ptr(ws), ws.numel(),
                             _stream(stream)))
    return out[:n]


SIGN_STATIC_MAX_POLYS = 262144


def sign_static(polys: DevicePolys, box, seed: int, k: int, cap: int, config: SignConfig | None = None,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """``sign`` on the library's static scratch (no workspace): int32 [n, k]."""
    check_device()
    n = polys.n
    if out is None:
        out = torch.empty((max(n, 1), k), dtype=torch.int32, device=polys.offsets.device)
    ps = polys.cstruct()
    cfg = ctypes.byref(config) if config is not None else None
    _check(lib().polymh_sign_static(ctypes.byref(ps), _box(box), seed & ((1 << 64) - 1), k, cap, _ptr(out), cfg,
                                    _stream(stream)))
    return out[:n]


def binned_params(polys: DevicePolys, box, k: int, cap: int, walk_ratio: float = 300.0,
                  max_bytes: int = 1 << 31):
    """(horizon, bin_bits) for sign_binned from the set's shape: the horizon
    covers about 16 expected first-hit indices N_B / N_P (Thm. 2) of the
    polygon at the 0.1% smallest area, within ``max_bytes`` of binned
    samples; the grid side puts about two cells across the median MBR side
    of the polygons the lookup signs (|B| / area >= ``walk_ratio``).  A
    host-side choice: the signatures do not depend on it."""
    mbr, area2, _ = prepare(polys)
    wx = float(box[2]) - float(box[0]) + 1.0
    wy = float(box[3]) - float(box[1]) + 1.0
    a_all = np.abs(area2.double().cpu().numpy()) / 2.0
    a = a_all[a_all > 0]
    if a.size == 0:
        return min(cap, 256), 0
    p_small = max(float(np.quantile(a, 0.001)) / (wx * wy), 1e-12)
    horizon = int(min(cap, 16.0 / p_small, max_bytes // (10 * k)))
    horizon = max(256, (horizon + 255) // 256 * 256) if horizon < cap else cap
    m = mbr.double().cpu().numpy()
    binned = (a_all > 0) & (wx * wy >= walk_ratio * a_all)
    if binned.any():
        m = m[binned]
    side = float(np.median(np.maximum(m[:, 2] - m[:, 0], m[:, 3] - m[:, 1]) + 1.0))
    bits = int(np.clip(np.round(np.log2(max(wx, wy) / max(side, 1.0))) + 1, 0, 6))
    return horizon, bits


def binned_config(polys: DevicePolys) -> SignConfig:
    """Launch shape for sign_binned: the default with an LDS edge cache just
    large enough for the set's largest polygon (64..1024 edges; larger
    polygons stream their edges), so more lookup workgroups share a CU.
    Synchronises once."""
    cnt = polys.offsets[1:] - polys.offsets[:-1]
    vmax = int(cnt.max().item()) if cnt.numel() else 0
    lds = 64
    while lds < min(vmax, 1024):
        lds *= 2
    return sign_config(lds_edges=lds)


def sign_binned_workspace_size(n: int, k: int, cap: int, horizon: int, bin_bits: int,
                               config: SignConfig | None = None) -> int:
    return int(lib().polymh_sign_binned_workspace_size(n, k, cap, horizon, bin_bits,
                                                       ctypes.byref(config) if config else None))


def sign_binned(polys: DevicePolys, box, seed: int, k: int, cap: int, horizon: int | None = None,
                bin_bits: int | None = None, walk_ratio: float = 300.0, config: SignConfig | None = None,
                out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                stream=None, rebin: bool = True) -> torch.Tensor:
    """Alg. 1 signatures from shared binned samples (equal to ``sign``'s, bit
    for bit).  ``horizon`` / ``bin_bits`` default to ``binned_params``;
    polygons with |B| / area below ``walk_ratio`` are walked instead.
    ``rebin=False`` reuses the bins already in ``ws`` from an earlier call
    with the same workspace and arguments (``polymh_sign_binned_prebinned``)."""
    check_device()
    if not rebin and ws is None:
        raise ValueError("sign_binned: rebin=False needs the workspace that holds the bins")
    dev = polys.offsets.device
    n = polys.n
    if horizon is None or bin_bits is None:
        h, b = binned_params(polys, box, k, cap, walk_ratio)
        horizon = h if horizon is None else horizon
        bin_bits = b if bin_bits is None else bin_bits
    if out is None:
        out = torch.empty((max(n, 1), k), dtype=torch.int32, device=dev)
    # zero for invalid arguments, which the call itself then reports
    need = max(sign_binned_workspace_size(n, k, cap, horizon, bin_bits, config), 256)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    ps = polys.cstruct()
    fn = lib().polymh_sign_binned if rebin else lib().polymh_sign_binned_prebinned
    _check(fn(ctypes.byref(ps), _box(box), seed & ((1 << 64) - 1), k, cap, horizon, bin_bits, float(walk_ratio),
              _ptr(out), ctypes.byref(config) if config else None, _ptr(ws), ws.numel(), _stream(stream)))
    return out[:n]


def band(sig: torch.Tensor, b: int, r: int, band_seed: int = 0, out: torch.Tensor | None = None,
         stream=None) -> torch.Tensor:
    """Band keys: int64 [N, b] holding uint64 values."""
    check_device()
    n, k = sig.shape
    if out is None:
        out = torch.empty((max(n, 1), b), dtype=torch.int64, device=sig.device)
    _check(lib().polymh_band(_ptr(sig), n, k, b, r, band_seed & ((1 << 64) - 1), _ptr(out),
                             _stream(stream)))
    return out[:n]


def index_build(keys: torch.Tensor, stream=None, ws: torch.Tensor | None = None):
    """Bucket table: (sorted_keys int64 [N*b], sorted entries int32 [N*b],
    entry = p*b + t)."""
    check_device()
    n, b = keys.shape
    dev = keys.device
    m = max(n * b, 1)
    sk = torch.empty(m, dtype=torch.int64, device=dev)
    si = torch.empty(m, dtype=torch.int32, device=dev)
    need = int(lib().polymh_index_workspace_size(n, b))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    _check(lib().polymh_index_build(_ptr(keys), n, b, _ptr(ws), ws.numel(), _ptr(sk), _ptr(si),
                                    _stream(stream)))
    return sk[:n * b], si[:n * b]


def query(sorted_keys: torch.Tensor, sorted_ids: torch.Tensor, n_data: int, qkeys: torch.Tensor,
          stream=None, ws: torch.Tensor | None = None):
    """Candidates: (cand_off int64 [nq+1], cand_ids int32 [C]); synchronises
    once to size cand_ids."""
    check_device()
    nq, b = qkeys.shape
    dev = qkeys.device
    need = int(lib().polymh_query_workspace_size(n_data, nq))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    off = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    s = _stream(stream)
    L = lib()
    _check(L.polymh_query(_ptr(sorted_keys), _ptr(sorted_ids), sorted_keys.numel(), n_data,
                          _ptr(qkeys), nq, b, _ptr(ws), ws.numel(), _ptr(off), None, 0, s))
    total = int(off[-1].item())
    ids = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
    _check(L.polymh_query(_ptr(sorted_keys), _ptr(sorted_ids), sorted_keys.numel(), n_data,
                          _ptr(qkeys), nq, b, _ptr(ws), ws.numel(), _ptr(off), _ptr(ids), -1, s))
    return off, ids[:total]


def refine_workspace(device="cuda") -> torch.Tensor:
    """A workspace for ``refine`` (heavy pairs split over many wavefronts)."""
    return _workspace(int(lib().polymh_refine_workspace_size()), device)


def refine(data: DevicePolys, queries: DevicePolys, cand_off: torch.Tensor, cand_ids: torch.Tensor,
           out: torch.Tensor | None = None, stream=None, n_cand: int | None = None,
           ws: torch.Tensor | None = None, split_heavy: bool = True) -> torch.Tensor:
    """Exact Jaccard per candidate: float64 [C] (C = n_cand, default the
    length of cand_ids; ranges come from cand_off on the device).  With
    ``split_heavy`` (``polymh_refine_ws``) very large pairs are spread over
    many wavefronts; ``ws`` defaults to a fresh workspace."""
    check_device()
    nq = queries.n
    c = cand_ids.numel() if n_cand is None else n_cand
    if out is None:
        out = torch.empty(max(c, 1), dtype=torch.float64, device=cand_ids.device)
    dp, qp = data.cstruct(), queries.cstruct()
    if not split_heavy:
        _check(lib().polymh_refine(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                   nq, c, _ptr(out), _stream(stream)))
        return out[:c]
    if ws is None:
        ws = refine_workspace(cand_ids.device)
    _check(lib().polymh_refine_ws(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                  nq, c, _ptr(out), None, _ptr(ws), ws.numel(), _stream(stream)))
    return out[:c]


def refine_stats(data: DevicePolys, queries: DevicePolys, cand_off, cand_ids, stream=None,
                 split_heavy: bool = True):
    """(J float64 [C], work counts: tiled pairs, edge pairs swept by the tiled form,
    general edge pairs, disjoint pairs)."""
    c = cand_ids.numel()
    out = torch.empty(max(c, 1), dtype=torch.float64, device=cand_ids.device)
    stats = torch.zeros(4, dtype=torch.int64, device=cand_ids.device)
    dp, qp = data.cstruct(), queries.cstruct()
    if split_heavy:
        ws = refine_workspace(cand_ids.device)
        _check(lib().polymh_refine_ws(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                      queries.n, c, _ptr(out), _ptr(stats), _ptr(ws), ws.numel(),
                                      _stream(stream)))
    else:
        _check(lib().polymh_refine_stats(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                         queries.n, c, _ptr(out), _ptr(stats), _stream(stream)))
    return out[:c], [int(v) for v in stats.cpu().tolist()]


def topk(cand_off: torch.Tensor, cand_ids: torch.Tensor, cand_j: torch.Tensor, k: int, stream=None,
         out=None):
    """(top_ids int32 [nq, k] (-1 pad), top_j float64 [nq, k])."""
    check_device()
    nq = cand_off.numel() - 1
    dev = cand_off.device
    if out is not None:
        ids, js = out
    else:
        ids = torch.empty((max(nq, 1), k), dtype=torch.int32, device=dev)
        js = torch.empty((max(nq, 1), k), dtype=torch.float64, device=dev)
    _check(lib().polymh_topk(_ptr(cand_off), _ptr(cand_ids), _ptr(cand_j), nq, k, _ptr(ids), _ptr(js),
                             _stream(stream)))
    return ids[:nq], js[:nq]


# ------------------------------------------------------------- scorer calls

def mlp_param_count() -> int:
    return int(lib().polymh_mlp_param_count())


def mlp_bf16_count() -> int:
    return int(lib().polymh_mlp_bf16_count())


def mlp_sync_bf16(params: torch.Tensor, wbf16: torch.Tensor, stream=None):
    _check(lib().polymh_mlp_sync_bf16(_ptr(params), _ptr(wbf16), _stream(stream)))


def mlp_buffers(B: int, device="cuda"):
    """(acts, scratch) byte buffers for batch B."""
    L = lib()
    return (_workspace(L.polymh_mlp_acts_size(B), device),
            _workspace(L.polymh_mlp_scratch_size(B), device))


def mlp_forward(X: torch.Tensor, params, wbf16, acts, y=None, stream=None):
    """X: int16 [B, 288] (BF16 bits), B a multiple of 32 -> y float32 [B]."""
    B = X.shape[0]
    if y is None:
        y = torch.empty(max(B, 1), dtype=torch.float32, device=X.device)
    _check(lib().polymh_mlp_forward(_ptr(X), B, _ptr(params), _ptr(wbf16), _ptr(y), _ptr(acts),
                                    acts.numel(), _stream(stream)))
    return y[:B]


def mlp_backward(X, params, wbf16, acts, label, grad, loss, scratch, stream=None):
    _check(lib().polymh_mlp_backward(_ptr(X), X.shape[0], _ptr(params), _ptr(wbf16), _ptr(acts),
                                     acts.numel(), _ptr(label), _ptr(grad), _ptr(loss),
                                     _ptr(scratch), scratch.numel(), _stream(stream)))


def mlp_adam(params, grad, m, v, step, wbf16, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().polymh_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2,
                                 eps, _ptr(wbf16), _stream(stream)))


def gemm_bf16(A, a_row_stride, a_k_stride, B, b_col_stride, b_k_stride, M, N, K, stream=None):
    C = torch.empty((max(M, 1), max(N, 1)), dtype=torch.float32, device=A.device)
    _check(lib().polymh_gemm_bf16(_ptr(A), a_row_stride, a_k_stride, _ptr(B), b_col_stride,
                                  b_k_stride, M, N, K, _ptr(C), _stream(stream)))
    return C[:M, :N]


def poly_features(polys: DevicePolys, box, out=None, stream=None) -> torch.Tensor:
    f = torch.empty((max(polys.n, 1), 12), dtype=torch.float32, device=polys.offsets.device) if out is None else out
    ps = polys.cstruct()
    _check(lib().polymh_poly_features(ctypes.byref(ps), _box(box), _ptr(f), _stream(stream)))
    return f[:polys.n]


def pair_features(lsig, lfeat, rsig, rfeat, li, ri, R_pad=None, out=None, stream=None):
    R = li.numel()
    R_pad = R if R_pad is None else R_pad
    if out is None:
        out = torch.empty((max(R_pad, 1), 288), dtype=torch.int16, device=lsig.device)
    _check(lib().polymh_pair_features(_ptr(lsig), _ptr(lfeat), _ptr(rsig), _ptr(rfeat),
                                      lsig.shape[1], _ptr(li), _ptr(ri), R, R_pad, _ptr(out),
                                      _stream(stream)))
    return out[:R_pad]


def csr_rows(cand_off, n_cand, stream=None):
    rows = torch.empty(max(n_cand, 1), dtype=torch.int32, device=cand_off.device)
    _check(lib().polymh_csr_rows(_ptr(cand_off), cand_off.numel() - 1, _ptr(rows), _stream(stream)))
    return rows[:n_cand]


def jhat(lsig, rsig, li, ri, out=None, stream=None):
    R = li.numel()
    if out is None:
        out = torch.empty(max(R, 1), dtype=torch.float32, device=lsig.device)
    _check(lib().polymh_jhat(_ptr(lsig), _ptr(rsig), lsig.shape[1], _ptr(li), _ptr(ri), R, _ptr(out),
                             _stream(stream)))
    return out[:R]


def rank_head(cand_off, cand_ids, score, M, stream=None):
    """Per query, the first min(M, C_q) candidates by decreasing score:
    (head_off int64 [nq+1], head_query int32, head_cand int64, head_id int32)."""
    nq = cand_off.numel() - 1
    dev = cand_off.device
    C = score.numel()
    order = torch.empty(max(C, 1), dtype=torch.int32, device=dev)
    ok = torch.empty(max(nq, 1), dtype=torch.uint8, device=dev)
    hoff = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    hq = torch.empty(max(nq * M, 1), dtype=torch.int32, device=dev)
    hc = torch.empty(max(nq * M, 1), dtype=torch.int64, device=dev)
    hid = torch.empty(max(nq * M, 1), dtype=torch.int32, device=dev)
    _check(lib().polymh_rank_head(_ptr(cand_off), _ptr(cand_ids), nq, _ptr(score), M, _ptr(order),
                                  _ptr(ok), _ptr(hoff), _ptr(hq), _ptr(hc), _ptr(hid), _stream(stream)))
    return hoff, hq, hc, hid


def scatter_scores(idx, val, score, stream=None):
    _check(lib().polymh_scatter_scores(_ptr(idx), _ptr(val), idx.numel(), _ptr(score), _stream(stream)))


def rank_refine(data: DevicePolys, queries: DevicePolys, cand_off, cand_ids, score, topk=10, F=16,
                margin=0.0, max_rounds=1 << 20, ws=None, stream=None):
    """Best-first refinement with early stop -> (top_ids, top_j, n_refined, rounds)."""
    nq = queries.n
    C = cand_ids.numel()
    dev = cand_off.device
    need = int(lib().polymh_rank_workspace_size(nq, C, F))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    ids = torch.empty((max(nq, 1), topk), dtype=torch.int32, device=dev)
    js = torch.empty((max(nq, 1), topk), dtype=torch.float64, device=dev)
    nref = ctypes.c_int64(0)
    rounds = ctypes.c_int32(0)
    dp, qp = data.cstruct(), queries.cstruct()
    _check(lib().polymh_rank_refine(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                    _ptr(score), nq, C, topk, F, float(margin), max_rounds, _ptr(ws),
                                    ws.numel(), _ptr(ids), _ptr(js), ctypes.byref(nref),
                                    ctypes.byref(rounds), _stream(stream)))
    return ids[:nq], js[:nq], int(nref.value), int(rounds.value)


def sig_pack(sig, out=None, stream=None):
    """The saturated signature table of sig [n][k] (k a multiple of 4 up to
    256): uint16 bit patterns in an int16 tensor [n][k], min(value, 65535)."""
    n, k = sig.shape
    if int(lib().polymh_sig_pack_stride(k)) == 0:
        raise ValueError("the saturated signature table needs k a multiple of 4 in [4, 256]")
    out = torch.empty((max(n, 1), k), dtype=torch.int16, device=sig.device) if out is None else out
    _check(lib().polymh_sig_pack(_ptr(sig), n, k, _ptr(out), _stream(stream)))
    return out


def rank_jhat_order(qsig, dsig, cand_off, cand_ids, score=None, order=None, sorted_ok=None, stream=None,
                    packed=None):
    """Collision fraction of every candidate and each query's best-first
    order: (score float32 [C], order int32 [C], sorted_ok uint8 [nq]).  With
    ``packed`` (``sig_pack(dsig)``) the candidates are read from the
    saturated table; the result is the same."""
    nq = cand_off.numel() - 1
    dev = cand_off.device
    C = cand_ids.numel()
    score = torch.empty(max(C, 1), dtype=torch.float32, device=dev) if score is None else score
    order = torch.empty(max(C, 1), dtype=torch.int32, device=dev) if order is None else order
    sorted_ok = torch.empty(max(nq, 1), dtype=torch.uint8, device=dev) if sorted_ok is None else sorted_ok
    if packed is not None:
        _check(lib().polymh_rank_jhat_order_packed(_ptr(qsig), _ptr(packed), _ptr(dsig), qsig.shape[1],
                                                   _ptr(cand_off), _ptr(cand_ids), nq, _ptr(score), _ptr(order),
                                                   _ptr(sorted_ok), _stream(stream)))
    else:
        _check(lib().polymh_rank_jhat_order(_ptr(qsig), _ptr(dsig), qsig.shape[1], _ptr(cand_off),
                                            _ptr(cand_ids), nq, _ptr(score), _ptr(order), _ptr(sorted_ok),
                                            _stream(stream)))
    return score, order, sorted_ok


def rank_order(cand_off, score, order, sorted_ok, stream=None):
    """Best-first order of each query's candidates by the given scores."""
    _check(lib().polymh_rank_order(_ptr(cand_off), cand_off.numel() - 1, _ptr(score), _ptr(order),
                                   _ptr(sorted_ok), _stream(stream)))


def rank_head_fixed(cand_off, cand_ids, order, M, out=None, stream=None):
    """First M candidates of each query's order in fixed slots q*M + t:
    (head_query int32, head_cand int64 (-1 empty), head_id int32 (-1 empty))."""
    nq = cand_off.numel() - 1
    dev = cand_off.device
    if out is None:
        n = max(nq * M, 1)
        out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int64, device=dev),
               torch.empty(n, dtype=torch.int32, device=dev))
    hq, hc, hid = out
    _check(lib().polymh_rank_head_fixed(_ptr(cand_off), _ptr(cand_ids), nq, _ptr(order), M, _ptr(hq), _ptr(hc),
                                        _ptr(hid), _stream(stream)))
    return hq, hc, hid


def rank_reorder_head(cand_off, score, order_in, M, sorted_ok, order_out, stream=None):
    """Order after the first M candidates of each query got new scores."""
    _check(lib().polymh_rank_reorder_head(_ptr(cand_off), cand_off.numel() - 1, _ptr(score), _ptr(order_in), M,
                                          _ptr(sorted_ok), _ptr(order_out), _stream(stream)))


def mlp_score_pairs(lsig, lfeat, rsig, rfeat, li, ri, params, wbf16, out=None, out_idx=None, stream=None):
    """Fused scorer inference for pairs (li[r], ri[r]): float32 predictions
    in out[r], or in out[out_idx[r]] when out_idx is given."""
    R = li.numel()
    if out is None:
        out = torch.empty(max(R, 1), dtype=torch.float32, device=li.device)
    _check(lib().polymh_mlp_score_pairs(_ptr(lsig), _ptr(lfeat), _ptr(rsig), _ptr(rfeat), lsig.shape[1], _ptr(li),
                                        _ptr(ri), _ptr(out_idx), R, _ptr(params), _ptr(wbf16), _ptr(out),
                                        _stream(stream)))
    return out


def rank_refine_ordered(data: DevicePolys, queries: DevicePolys, cand_off, cand_ids, score, order, sorted_ok,
                        topk=10, F=16, rounds=4, margin=0.0, ws=None, out=None, counts=None, n_cand=None,
                        stream=None):
    """Best-first refinement with early stop and no host reads (graph-
    capturable): (top_ids, top_j, counts int64 [2] = refined pairs, queries
    completed by the finishing pass)."""
    nq = queries.n
    C = cand_ids.numel() if n_cand is None else n_cand
    dev = cand_off.device
    need = int(lib().polymh_rank_workspace_size(nq, C, F))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    if out is None:
        out = (torch.empty((max(nq, 1), topk), dtype=torch.int32, device=dev),
               torch.empty((max(nq, 1), topk), dtype=torch.float64, device=dev))
    ids, js = out
    counts = torch.zeros(2, dtype=torch.int64, device=dev) if counts is None else counts
    dp, qp = data.cstruct(), queries.cstruct()
    _check(lib().polymh_rank_refine_ordered(ctypes.byref(dp), ctypes.byref(qp), _ptr(cand_off), _ptr(cand_ids),
                                            _ptr(score), _ptr(order), _ptr(sorted_ok), nq, C, topk, F, rounds,
                                            float(margin), _ptr(ws), ws.numel(), _ptr(ids), _ptr(js),
                                            _ptr(counts), _stream(stream)))
    return ids[:nq], js[:nq], counts


def rank_workspace(nq, n_cand, F, device="cuda"):
    return _workspace(int(lib().polymh_rank_workspace_size(nq, n_cand, F)), device)


# ------------------------------------------------------- graphs (batching)

def query_capped(sorted_keys, sorted_ids, n_data, qkeys, cand_off, cand_ids, overflow, ws, stream=None):
    """Both lookup phases with a fixed capacity and a device overflow flag."""
    nq, b = qkeys.shape
    _check(lib().polymh_query_capped(_ptr(sorted_keys), _ptr(sorted_ids), sorted_keys.numel(), n_data,
                                     _ptr(qkeys), nq, b, _ptr(ws), ws.numel(), _ptr(cand_off),
                                     _ptr(cand_ids), cand_ids.numel(), _ptr(overflow), _stream(stream)))


class Graph:
    """A captured sequence of libpolymh calls; replay with launch()."""

    def __init__(self, handle, stream):
        self.handle = handle
        self.stream = stream

    def launch(self, stream=None):
        _check(lib().polymh_graph_launch(self.handle, _stream(stream or self.stream)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.polymh_graph_destroy(self.handle)
            self.handle = None


def capture(fn, stream):
    """Run fn() with every libpolymh call recorded on `stream` (a
    torch.cuda.Stream that fn must use) and return the instantiated graph."""
    _check(lib().polymh_graph_begin(_stream(stream)))
    try:
        with torch.cuda.stream(stream):
            fn()
    finally:
        h = ctypes.c_void_p()
        st = lib().polymh_graph_end(_stream(stream), ctypes.byref(h))
    _check(st)
    return Graph(h, stream)
