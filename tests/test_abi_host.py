"""Host-side checks of the C-ABI (no GPU): the library loads, exports every
function include/tdgemm.h declares, its structs have the layout the binding
assumes, and invalid descriptors are rejected on the host before any launch."""
import ctypes
import math
import pathlib
import re
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "tdgemm.h"


@pytest.fixture(scope="module")
def lib():
    so = ROOT / "paper_1110_5765_amd" / "libtdgemm.so"
    if not so.exists():
        from paper_1110_5765_amd import build
        build.build()
    return ctypes.CDLL(str(so))


@pytest.fixture(scope="module")
def binding(lib):
    from paper_1110_5765_amd import tdgemm
    return tdgemm


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdgemm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for need in ["tdgemm_plan", "tdgemm_compand", "tdgemm_pack", "tdgemm_gemm", "tdgemm_unpack"]:
        assert need in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    nm = subprocess.run(["nm", "-D", "--defined-only", str(ROOT / "paper_1110_5765_amd" / "libtdgemm.so")],
                        capture_output=True, text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", nm), n


def test_struct_layout_matches_binding(binding, tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tdgemm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(tdgemm_desc), sizeof(tdgemm_pair), sizeof(tdgemm_block_stats),'
                   'sizeof(tdgemm_calib), offsetof(tdgemm_desc, snr_db), offsetof(tdgemm_desc, accel),'
                   'offsetof(tdgemm_pair, w), offsetof(tdgemm_desc, w_allowed));return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(binding.Desc), ctypes.sizeof(binding.Pair), ctypes.sizeof(binding.BlockStats),
            ctypes.sizeof(binding.Calib), binding.Desc.snr_db.offset, binding.Desc.accel.offset,
            binding.Pair.w.offset, binding.Desc.w_allowed.offset]
    assert got == want
    assert binding.PAIR_DTYPE.itemsize == ctypes.sizeof(binding.Pair)
    assert binding.STATS_DTYPE.itemsize == ctypes.sizeof(binding.BlockStats)


def _desc(binding, **kw):
    d = binding.Desc()
    d.M, d.N, d.K = 256, 256, 256
    d.lda = d.ldb = d.ldc = 256
    d.in_dtype = d.prec = binding.F64
    d.L = 64
    d.form = binding.SYM
    d.ctrl = binding.CTRL_SNR
    d.w_allowed = binding.w_mask((1, 2, 4))
    d.fixed_w = 2
    d.snr_db = 40.0
    d.fixed_rmax = 2.0 ** 20
    d.sep_q = 127.0
    d.u_safe = 50.0
    for k, v in kw.items():
        if k == "accel_units":
            v = (ctypes.c_int32 * 5)(*v)
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    ({}, 0),
    ({"L": 96}, 0), ({"L": 96, "w_allowed": 2 | 4 | 8}, 0), ({"L": 96, "w_allowed": 2 | 4 | 8 | 16}, 0),
    ({"L": 80}, -2), ({"L": 0}, -1), ({"L": 128, "w_allowed": 2 | 8}, -1),
    ({"form": 3}, -1), ({"prec": 7}, -1),
    ({"in_dtype": 0, "prec": 1}, -2), ({"M": -1}, -1), ({"lda": 100}, -1), ({"ldc": 10}, -1),
    ({"trans_a": 2}, -1), ({"w_allowed": 4}, -1), ({"w_allowed": 2 | 8}, -1),
    ({"w_allowed": 2 | 32}, -1), ({"ctrl": 9}, -1), ({"snr_db": math.nan}, -1),
    ({"ctrl": 1, "fixed_w": 3}, -1), ({"ctrl": 1, "fixed_w": 3, "L": 96}, 0),
    ({"ctrl": 1, "fixed_w": 4, "L": 96}, 0), ({"ctrl": 2, "fixed_w": 3, "L": 96}, 0),
    ({"ctrl": 1, "fixed_w": 5}, -1), ({"ctrl": 1, "fixed_rmax": 0.0}, -1),
    ({"ctrl": 2, "sep_q": 0.5}, -1), ({"u_safe": 0.0}, -1), ({"K": 64 * 513, "lda": 64 * 513}, -2),
    ({"ctrl": 4}, 0), ({"ctrl": 4, "snr_db": -math.inf}, -1), ({"ctrl": 4, "fixed_rmax": -1.0}, -1),
    ({"ctrl": 4, "fixed_w": 3}, -1), ({"ctrl": 4, "snr_db": math.inf}, 0),
    ({"k_split": -1}, -1), ({"k_split": 3}, 0), ({"k_split": 1000}, 0),
    # L * lda or L * ldb at 2^30 bytes and above: beyond the fused kernel's 32-bit
    # buffer offsets (FP64 elements of 8 bytes, FP32 of 4)
    ({"lda": (1 << 30) // (64 * 8)}, -2), ({"lda": (1 << 30) // (64 * 8) - 1}, 0),
    ({"ldb": (1 << 30) // (128 * 8), "L": 128}, -2), ({"ldb": (1 << 30) // (128 * 8) - 1, "L": 128}, 0),
    ({"ldb": (1 << 30) // (128 * 4), "L": 128, "in_dtype": 1, "prec": 1}, -2),
    ({"ldb": (1 << 30) // (128 * 4) - 1, "L": 128, "in_dtype": 1, "prec": 1}, 0),
    # measured saved-time units of the throughput control (Sec. 5.B F_W)
    ({"ctrl": 3, "accel": 0.5, "accel_units": (0, 0, 1365, 0, 2000)}, 0),
    ({"ctrl": 3, "accel_units": (0, 7, 1365, 0, 2000)}, -1), ({"ctrl": 3, "accel_units": (0, 0, -1, 0, 0)}, -1),
    ({"ctrl": 3, "accel_units": (0, 0, 1 << 21, 0, 0)}, -1), ({"accel_units": (0, 7, 0, 0, 0)}, 0),
])
def test_descriptor_validation(binding, lib, kw, status):
    d = _desc(binding, **kw)
    size = lib.tdgemm_workspace_size
    size.restype = ctypes.c_size_t
    n = size(ctypes.byref(d))
    assert (n > 0) == (status == 0)
    h = ctypes.c_void_p()
    # invalid descriptors are rejected before anything touches the GPU
    if status != 0:
        st = lib.tdgemm_plan(ctypes.byref(d), None, None, None, None, ctypes.c_size_t(0), None, ctypes.byref(h))
        assert st == status
        assert not h.value


@pytest.mark.parametrize("ctrl,values,status", [
    (0, [30.0, math.inf, -5.0, 80.0], 0), (0, [30.0, math.nan, 20.0, 20.0], -1),
    (3, [0.0, 1.0, 0.5, 0.25], 0), (3, [0.5, 1.5, 0.5, 0.5], -1), (3, [0.5, -0.1, 0.5, 0.5], -1),
    (1, [30.0, 30.0, 30.0, 30.0], -1), (2, [30.0, 30.0, 30.0, 30.0], -1),
    (4, [30.0, math.inf, 10.0, 80.0], 0), (4, [30.0, -math.inf, 10.0, 80.0], -1)])
def test_tile_target_validation(binding, lib, ctrl, values, status):
    """Per-inner-kernel targets (2 x 2 inner kernels): checked on the host."""
    d = _desc(binding, M=128, N=100, ctrl=ctrl, ldc=100)
    arr = (ctypes.c_double * 4)(*values)
    d.tile_target = ctypes.cast(arr, ctypes.c_void_p).value
    size = lib.tdgemm_workspace_size
    size.restype = ctypes.c_size_t
    assert (size(ctypes.byref(d)) > 0) == (status == 0)
    if status != 0:
        h = ctypes.c_void_p()
        assert lib.tdgemm_plan(ctypes.byref(d), None, None, None, None, ctypes.c_size_t(0), None,
                               ctypes.byref(h)) == status


def test_plan_rejects_missing_workspace_and_calibration(binding, lib):
    d = _desc(binding)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the checks fail first
    st = lib.tdgemm_plan(ctypes.byref(d), dummy, dummy, None, None, ctypes.c_size_t(0), None, ctypes.byref(h))
    assert st == -3
    need = binding.tdgemm_workspace_size(d)
    st = lib.tdgemm_plan(ctypes.byref(d), dummy, dummy, None, dummy, ctypes.c_size_t(need - 1), None, ctypes.byref(h))
    assert st == -3
    st = lib.tdgemm_plan(ctypes.byref(d), dummy, dummy, None, dummy, ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == -4                    # SNR control without a calibration table
    bad = binding.Calib(0, 0x1000, 0x1000)
    st = lib.tdgemm_plan(ctypes.byref(d), dummy, dummy, ctypes.byref(bad), dummy, ctypes.c_size_t(need), None,
                         ctypes.byref(h))
    assert st == -4


def test_calibrate_argument_errors(binding, lib):
    lib.tdgemm_calibrate_workspace_size.restype = ctypes.c_size_t
    assert lib.tdgemm_calibrate_workspace_size(80, 5) == 0
    assert lib.tdgemm_calibrate_workspace_size(64, 5) > 0
    assert lib.tdgemm_calibrate_workspace_size(96, 5) > 0
    f = lib.tdgemm_calibrate
    z = ctypes.c_void_p(0x1000)
    q = (ctypes.c_double * 1)(0.5)    # q < 1 is rejected
    out = (ctypes.c_double * 1)()
    assert f(64, 2, 1, 0, q, 1, z, z, 5, ctypes.c_double(50.0), out, out, out, z, ctypes.c_size_t(1 << 30), None) == -1
    q[0] = 4.0
    assert f(64, 3, 1, 0, q, 1, z, z, 5, ctypes.c_double(50.0), out, out, out, z, ctypes.c_size_t(1 << 30), None) == -1
    # W = 4 at L = 96 is a valid packing: the (too small) workspace is what fails
    assert f(96, 4, 1, 0, q, 1, z, z, 5, ctypes.c_double(50.0), out, out, out, z, ctypes.c_size_t(16), None) == -3
    assert f(80, 2, 1, 0, q, 1, z, z, 5, ctypes.c_double(50.0), out, out, out, z, ctypes.c_size_t(1 << 30), None) == -2
    assert f(64, 2, 1, 0, q, 1, z, z, 5, ctypes.c_double(50.0), out, out, out, z, ctypes.c_size_t(16), None) == -3


def test_status_strings(lib):
    f = lib.tdgemm_status_string
    f.restype = ctypes.c_char_p
    for s in (0, -1, -2, -3, -4, -5):
        assert f(s).decode().startswith("TDGEMM_")


def test_matrix_layout_detection(binding):
    import torch
    X = torch.zeros(5, 7)
    assert binding.matrix_layout(X) == (0, 7)
    assert binding.matrix_layout(X.t()) == (1, 7)
    Y = torch.zeros(6, 10)[:, :4]
    assert binding.matrix_layout(Y) == (0, 10)
    with pytest.raises(ValueError):
        binding.matrix_layout(torch.zeros(4, 6)[:, ::2])


def test_k_split_workspace(binding, lib):
    """A split l-sum keeps ceil(nL / s) partial M x N results in the workspace."""
    size = lib.tdgemm_workspace_size
    size.restype = ctypes.c_size_t
    d1 = _desc(binding, K=64 * 10, lda=64 * 10)
    d4 = _desc(binding, K=64 * 10, lda=64 * 10, k_split=4)          # groups of 3: 4 groups
    extra = size(ctypes.byref(d4)) - size(ctypes.byref(d1))
    assert 4 * 256 * 256 * 8 <= extra < 4 * 256 * 256 * 8 + 512
    d8 = _desc(binding, prec=binding.I8, ctrl=binding.CTRL_SEPARABLE, fixed_w=1, L=128, k_split=2)
    assert size(ctypes.byref(d8)) == 0


def test_plan_query_rejects_null_plan(lib):
    f = lib.tdgemm_plan_query
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_int64)]
    snr, short = ctypes.c_double(1.0), ctypes.c_int64(5)
    assert f(None, ctypes.byref(snr), None, ctypes.byref(short)) == -1


def test_noalloc_rejections_before_any_launch(binding, lib):
    """tdgemm_matmul_noalloc checks on the host, before touching a device: an
    invalid descriptor, a tile map or a block-scaled form, a workspace beyond the
    static array, a missing calibration table."""
    f = lib.tdgemm_matmul_noalloc
    f.restype = ctypes.c_int32
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the checks fail first
    cal = binding.Calib(1, 0x1000, 0x1000)

    def call(d, calib=cal):
        return f(ctypes.byref(d), dummy, dummy, ctypes.byref(calib) if calib is not None else None, dummy,
                 None)

    assert call(_desc(binding, M=-1)) == -1
    d = _desc(binding)
    nI = nJ = 256 // 64
    tmap = (ctypes.c_double * (nI * nJ))(*([30.0] * (nI * nJ)))
    d.tile_target = ctypes.cast(tmap, ctypes.c_void_p)
    assert call(d) == -2
    assert call(_desc(binding, prec=binding.I8, ctrl=binding.CTRL_SEPARABLE, fixed_w=1, L=128)) == -2
    big = _desc(binding, M=4096, N=4096, K=4096, lda=4096, ldb=4096, ldc=4096, k_split=64)
    assert binding.tdgemm_workspace_size(big) > binding.NOALLOC_MAX_BYTES
    assert call(big) == -3
    assert call(_desc(binding), None) == -4
