"""Python binding of the tdgemm C-ABI (include/tdgemm.h): argument marshalling only.

Every function takes torch tensors that live on the current HIP device,
passes their data pointers, sizes and the current stream to the library, and
converts status codes to exceptions. No arithmetic of the method happens here:
every step runs in the library's HIP kernels. The library is loaded from this
package's directory; if it is missing, import fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import pathlib

import numpy as np
import torch

LIB_PATH = pathlib.Path(__file__).resolve().parent / "libtdgemm.so"

F64, F32, I8, E4M3 = 0, 1, 2, 3
SYM, ASYM = 1, 2
CTRL_SNR, CTRL_FIXED, CTRL_SEPARABLE, CTRL_ACCEL, CTRL_TARGET = 0, 1, 2, 3, 4
STATUS = {0: "TDGEMM_OK", -1: "TDGEMM_E_ARG", -2: "TDGEMM_E_UNSUPPORTED",
          -3: "TDGEMM_E_WORKSPACE", -4: "TDGEMM_E_CALIB", -5: "TDGEMM_E_HIP"}
FORMS = {"sym": SYM, "asym": ASYM}
PRECS = {"f64": F64, "f32": F32, "i8": I8, "e4m3": E4M3}
CTRLS = {"snr": CTRL_SNR, "fixed": CTRL_FIXED, "separable": CTRL_SEPARABLE, "accel": CTRL_ACCEL,
         "target": CTRL_TARGET}


class Desc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("trans_a", ctypes.c_int32), ("trans_b", ctypes.c_int32),
                ("in_dtype", ctypes.c_int32), ("prec", ctypes.c_int32), ("L", ctypes.c_int32),
                ("form", ctypes.c_int32), ("ctrl", ctypes.c_int32), ("w_allowed", ctypes.c_uint32),
                ("fixed_w", ctypes.c_int32), ("snr_db", ctypes.c_double),
                ("fixed_rmax", ctypes.c_double), ("sep_q", ctypes.c_double),
                ("u_safe", ctypes.c_double), ("accel", ctypes.c_double),
                ("tile_target", ctypes.c_void_p), ("k_split", ctypes.c_int32),
                ("accel_units", ctypes.c_int32 * 5)]


class Calib(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("r", ctypes.c_void_p), ("s", ctypes.c_void_p)]


class BlockStats(ctypes.Structure):
    _fields_ = [("mn", ctypes.c_double), ("mx", ctypes.c_double), ("sumsq", ctypes.c_double),
                ("n", ctypes.c_int64)]


class Pair(ctypes.Structure):
    _fields_ = [("c_a", ctypes.c_double), ("c_b", ctypes.c_double), ("inv", ctypes.c_double),
                ("d", ctypes.c_double), ("r_max", ctypes.c_double), ("s_rep", ctypes.c_double),
                ("q_a", ctypes.c_double), ("q_b", ctypes.c_double), ("w", ctypes.c_int32),
                ("p", ctypes.c_int32)]


STATS_DTYPE = np.dtype([("mn", "<f8"), ("mx", "<f8"), ("sumsq", "<f8"), ("n", "<i8")])
PAIR_DTYPE = np.dtype([("c_a", "<f8"), ("c_b", "<f8"), ("inv", "<f8"), ("d", "<f8"),
                       ("r_max", "<f8"), ("s_rep", "<f8"), ("q_a", "<f8"), ("q_b", "<f8"),
                       ("w", "<i4"), ("p", "<i4")])


class TdgemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


def _load() -> ctypes.CDLL:
    if not LIB_PATH.exists():
        raise ImportError(f"tdgemm HIP library not built: {LIB_PATH} is missing "
                          f"(run paper_1110_5765_amd/build.py)")
    lib = ctypes.CDLL(str(LIB_PATH))
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "tdgemm_workspace_size": (sz, [P(Desc)]),
        "tdgemm_plan": (i32, [P(Desc), vp, vp, P(Calib), vp, sz, vp, P(vp)]),
        "tdgemm_compand": (i32, [vp, vp, vp, vp, vp, vp]),
        "tdgemm_pack": (i32, [vp, vp, vp, vp, vp, vp]),
        "tdgemm_gemm": (i32, [vp, vp, vp, vp, ctypes.c_int, vp]),
        "tdgemm_unpack": (i32, [vp, vp, vp, vp, vp]),
        "tdgemm_plan_export": (i32, [vp, vp, vp, vp, vp]),
        "tdgemm_plan_dims": (i32, [vp, P(i64), P(i64), P(i64), P(i64)]),
        "tdgemm_plan_query": (i32, [vp, P(dbl), vp, P(i64)]),
        "tdgemm_plan_destroy": (i32, [vp]),
        "tdgemm_calibrate_workspace_size": (sz, [i32, i32]),
        "tdgemm_calibrate": (i32, [i32, i32, i32, i32, vp, i32, vp, vp, i32, dbl, vp, vp, vp,
                                   vp, sz, vp]),
        "tdgemm_matmul_noalloc": (i32, [P(Desc), vp, vp, P(Calib), vp, vp]),
        "tdgemm_status_string": (ctypes.c_char_p, [i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = _load()


def _check(status: int, where: str) -> None:
    if status != 0:
        raise TdgemmError(status, where)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def matrix_layout(X: torch.Tensor) -> tuple[int, int]:
    """(trans, ld) of a 2-D tensor that is row-major or the transpose of one."""
    if X.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    r, c = X.shape
    s0, s1 = X.stride()
    if s1 == 1 and (r <= 1 or s0 >= max(c, 1)):
        return 0, max(s0, c, 1)
    if s0 == 1 and (c <= 1 or s1 >= max(r, 1)):
        return 1, max(s1, r, 1)
    raise ValueError("matrix must be row-major or a transposed row-major view")


def w_mask(ws) -> int:
    m = 0
    for w in ws:
        m |= 1 << int(w)
    return m


def make_desc(A: torch.Tensor, B: torch.Tensor, *, L: int = 64, form: str = "sym",
              prec: str | None = None, ctrl: str = "snr", snr_db: float = 40.0,
              w_allowed=(1, 2, 4), fixed_w: int = 2, fixed_rmax: float = float(2 ** 20),
              sep_q: float = 127.0, u_safe: float = 50.0, accel: float = 1.0,
              ldc: int | None = None, tile_target=None, k_split: int = 1,
              accel_units: dict | None = None) -> Desc:
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    ta, lda = matrix_layout(A)
    tb, ldb = matrix_layout(B)
    d = Desc()
    d.M, d.N, d.K = M, N, K
    d.lda, d.ldb = lda, ldb
    d.ldc = max(N, 1) if ldc is None else ldc
    d.trans_a, d.trans_b = ta, tb
    d.in_dtype = _dtype_code(A)
    d.prec = d.in_dtype if prec is None else PRECS[prec]
    d.L = L
    d.form = FORMS[form]
    d.ctrl = CTRLS[ctrl]
    d.w_allowed = w_mask(w_allowed)
    d.fixed_w = fixed_w
    d.snr_db = snr_db
    d.fixed_rmax = fixed_rmax
    d.sep_q = sep_q
    d.u_safe = u_safe
    d.accel = accel
    d.k_split = k_split
    if accel_units is not None:           # {W: saved-time units} from measured F_W
        for w, u in accel_units.items():
            d.accel_units[int(w)] = int(u)
    if tile_target is not None:
        # host array nI x nJ of per-inner-kernel targets (S in dB or F_kernel); the
        # descriptor keeps it alive for tdgemm_plan
        nI, nJ = -(-M // L), -(-N // L)
        t = np.ascontiguousarray(np.asarray(tile_target, dtype=np.float64))
        if t.shape != (nI, nJ):
            raise ValueError(f"tile_target must be {nI} x {nJ}, got {t.shape}")
        d._tile_keep = t
        d.tile_target = t.ctypes.data
    return d


def auto_k_split(M: int, N: int, K: int, L: int, prec: str = "f64", cus: int = 256) -> int:
    """A k_split for products whose M and N leave fewer fused workgroups than
    CUs; 1 otherwise. With groups of g subblocks an inner kernel has
    ceil(nL / g) groups, and the launch runs ceil(tiles * groups / slots) rounds
    of workgroups that multiply g pairs each, where slots is the number of
    fused workgroups resident at once (one per CU at L = 96 and 128; at L = 64
    two for FP64 packing and three for FP32). A workgroup also costs about two
    pairs' time of its own (first loads, writing its partial tile), so the
    smallest rounds * (g + 2) wins, fewer groups on ties (less partial traffic
    for the ordered group sum). Only the order of the l-sum changes, in the way
    tdgemm_desc.k_split describes."""
    nI, nJ, nL = -(-M // L), -(-N // L), -(-K // L)
    tiles = max(1, nI * nJ)
    if nL <= 1 or tiles >= cus:
        return 1
    slots = cus * ((3 if prec == "f32" else 2) if L == 64 else 1)
    best = None
    for g in range(1, nL + 1):
        groups = -(-nL // g)
        rounds = -(-(tiles * groups) // slots)
        key = (rounds * (g + 2), groups)
        if best is None or key < best[0]:
            best = (key, groups)
    return best[1]


def torch_dtype(prec_code: int) -> torch.dtype:
    return torch.float64 if prec_code == F64 else torch.float32


class DeviceCalib:
    """s(R, W) table in device memory (see tdgemm_calib): r[n_r], s[3][n_r]."""

    def __init__(self, r: np.ndarray, s_by_w: dict, device="cuda"):
        r = np.asarray(r, dtype=np.float64)
        s = np.full((3, r.size), np.inf)
        for W, sw in s_by_w.items():
            s[W - 2] = np.asarray(sw, dtype=np.float64)
        self.r = torch.from_numpy(r.copy()).to(device)
        self.s = torch.from_numpy(s.ravel().copy()).to(device)
        self.struct = Calib(int(r.size), self.r.data_ptr(), self.s.data_ptr())


class Plan:
    """Owns a tdgemm_plan_t and keeps its workspace and calibration alive."""

    def __init__(self, handle: ctypes.c_void_p, desc: Desc, ws: torch.Tensor, calib, stream):
        self.handle = handle
        self.desc = desc
        self.ws = ws
        self.calib = calib
        self.stream = stream

    @property
    def dims(self):
        return tdgemm_plan_dims(self)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.tdgemm_plan_destroy(h)
            self.handle = None


def tdgemm_workspace_size(desc: Desc) -> int:
    return int(_LIB.tdgemm_workspace_size(ctypes.byref(desc)))


def tdgemm_plan(desc: Desc, A: torch.Tensor, B: torch.Tensor, calib: DeviceCalib | None = None,
                ws: torch.Tensor | None = None, stream=None) -> Plan:
    need = tdgemm_workspace_size(desc)
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=A.device)
    h = ctypes.c_void_p()
    cal = ctypes.byref(calib.struct) if calib is not None else None
    st = _stream(stream)
    _check(_LIB.tdgemm_plan(ctypes.byref(desc), _ptr(A), _ptr(B), cal, _ptr(ws), ws.numel(),
                            st, ctypes.byref(h)), "tdgemm_plan")
    return Plan(h, desc, ws, calib, st)


def tdgemm_compand(plan: Plan, A, B, qA, qB, stream=None) -> None:
    _check(_LIB.tdgemm_compand(plan.handle, _ptr(A), _ptr(B), _ptr(qA), _ptr(qB), _stream(stream)),
           "tdgemm_compand")


def tdgemm_pack(plan: Plan, qA, qB, pA, pB, stream=None) -> None:
    _check(_LIB.tdgemm_pack(plan.handle, _ptr(qA), _ptr(qB), _ptr(pA), _ptr(pB), _stream(stream)),
           "tdgemm_pack")


def tdgemm_gemm(plan: Plan, a, b, out, fused: int = 1, stream=None) -> None:
    _check(_LIB.tdgemm_gemm(plan.handle, _ptr(a), _ptr(b), _ptr(out), int(fused), _stream(stream)),
           "tdgemm_gemm")


def tdgemm_unpack(plan: Plan, Rbar, r_int, C, stream=None) -> None:
    _check(_LIB.tdgemm_unpack(plan.handle, _ptr(Rbar), _ptr(r_int), _ptr(C), _stream(stream)),
           "tdgemm_unpack")


def tdgemm_plan_dims(plan: Plan) -> tuple[int, int, int, int]:
    v = [ctypes.c_int64() for _ in range(4)]
    _check(_LIB.tdgemm_plan_dims(plan.handle, *[ctypes.byref(x) for x in v]), "tdgemm_plan_dims")
    return tuple(int(x.value) for x in v)


def tdgemm_plan_query(plan: Plan) -> tuple[float, np.ndarray, int]:
    """(predicted output SNR in dB, W histogram [5], TARGET pairs short of their target)."""
    snr = ctypes.c_double()
    hist = np.zeros(5, dtype=np.int64)
    short = ctypes.c_int64()
    _check(_LIB.tdgemm_plan_query(plan.handle, ctypes.byref(snr), hist.ctypes.data, ctypes.byref(short)),
           "tdgemm_plan_query")
    return float(snr.value), hist, int(short.value)


def tdgemm_plan_export(plan: Plan):
    """(stats_a [nI, nL], stats_b [nL, nJ], pairs [nI, nJ, nL], budgets [nI, nJ]) as numpy."""
    nI, nL, nJ, n_pairs = tdgemm_plan_dims(plan)
    sa = np.zeros(nI * nL, dtype=STATS_DTYPE)
    sb = np.zeros(nL * nJ, dtype=STATS_DTYPE)
    pr = np.zeros(n_pairs, dtype=PAIR_DTYPE)
    bu = np.zeros(nI * nJ, dtype=np.float64)
    _check(_LIB.tdgemm_plan_export(plan.handle, sa.ctypes.data, sb.ctypes.data, pr.ctypes.data,
                                   bu.ctypes.data), "tdgemm_plan_export")
    return sa.reshape(nI, nL), sb.reshape(nL, nJ), pr.reshape(nI, nJ, nL), bu.reshape(nI, nJ)


def tdgemm_calibrate_workspace_size(L: int, n_inst: int) -> int:
    return int(_LIB.tdgemm_calibrate_workspace_size(L, n_inst))


def tdgemm_calibrate(L: int, W: int, form: str, prec: str, q, u_a: torch.Tensor,
                     u_b: torch.Tensor, u_safe: float = 50.0, ws: torch.Tensor | None = None,
                     stream=None):
    """Representation-noise table on the GPU path: returns (r, m, s) numpy arrays."""
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    n_inst = u_a.shape[0]
    need = tdgemm_calibrate_workspace_size(L, n_inst)
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=u_a.device)
    r = np.zeros(q.size)
    m = np.zeros(q.size)
    s = np.zeros(q.size)
    _check(_LIB.tdgemm_calibrate(L, W, FORMS[form], PRECS[prec], q.ctypes.data, q.size,
                                 _ptr(u_a), _ptr(u_b), n_inst, u_safe, r.ctypes.data, m.ctypes.data,
                                 s.ctypes.data, _ptr(ws), ws.numel(), _stream(stream)),
           "tdgemm_calibrate")
    return r, m, s


NOALLOC_MAX_BYTES = 32 << 20


def tdgemm_matmul_noalloc(desc: Desc, A: torch.Tensor, B: torch.Tensor, calib: DeviceCalib | None,
                          C: torch.Tensor, stream=None) -> None:
    """tdgemm_plan + fused tdgemm_gemm with the library's static device workspace."""
    cal = ctypes.byref(calib.struct) if calib is not None else None
    _check(_LIB.tdgemm_matmul_noalloc(ctypes.byref(desc), _ptr(A), _ptr(B), cal, _ptr(C),
                                      _stream(stream)), "tdgemm_matmul_noalloc")


def tdgemm_status_string(status: int) -> str:
    return _LIB.tdgemm_status_string(status).decode()


# ---------------------------------------------------------------------------
def slot_elems(plan: Plan) -> int:
    """Elements of a per-pair staging buffer (n_pairs L x L slots)."""
    return plan.dims[3] * plan.desc.L * plan.desc.L


def block_scaled_shapes(plan: Plan) -> dict:
    """Buffer shapes of the block-scaled forms: byte operands qA ((nI L) x (nL L)),
    qB ((nJ L) x (nL L), B^T) and per-pair products (n_pairs x L x L)."""
    nI, nL, nJ, n_pairs = plan.dims
    L = plan.desc.L
    return {"qA": (nI * L, nL * L), "qB": (nJ * L, nL * L), "products": (n_pairs, L, L)}


def block_scaled_matmul(A: torch.Tensor, B: torch.Tensor, fmt: str = "i8", q: float | None = None,
                        *, out: torch.Tensor | None = None, stream=None):
    """C (float32) = A B in the INT8 / FP8 block-scaled form: tdgemm_plan (separable
    block scales), tdgemm_compand (byte operands) and the fused tdgemm_gemm.
    Returns (C, plan, qA, qB)."""
    q = (127.0 if fmt == "i8" else 448.0) if q is None else q
    desc = make_desc(A, B, L=128, prec=fmt, ctrl="separable", fixed_w=1, sep_q=q)
    plan = tdgemm_plan(desc, A, B, None, stream=stream)
    sh = block_scaled_shapes(plan)
    qA = torch.empty(sh["qA"], dtype=torch.uint8, device=A.device)
    qB = torch.empty(sh["qB"], dtype=torch.uint8, device=A.device)
    if out is None:
        out = torch.empty((desc.M, desc.N), dtype=torch.float32, device=A.device)
    if desc.M > 0 and desc.N > 0 and desc.K > 0:
        tdgemm_compand(plan, A, B, qA, qB, stream=stream)
    tdgemm_gemm(plan, qA if qA.numel() else None, qB if qB.numel() else None, out, fused=1,
                stream=stream)
    return out, plan, qA, qB


def matmul(A: torch.Tensor, B: torch.Tensor, calib: DeviceCalib | None = None, *,
           out: torch.Tensor | None = None, stream=None, **kw) -> tuple[torch.Tensor, Plan]:
    """C = A B through tdgemm_plan + the fused tdgemm_gemm. Keyword arguments as make_desc."""
    desc = make_desc(A, B, **kw)
    plan = tdgemm_plan(desc, A, B, calib if desc.ctrl in (CTRL_SNR, CTRL_ACCEL, CTRL_TARGET) else None,
                       stream=stream)
    if out is None:
        out = torch.empty((desc.M, desc.N), dtype=torch_dtype(desc.prec), device=A.device)
    tdgemm_gemm(plan, A, B, out, fused=1, stream=stream)
    return out, plan
