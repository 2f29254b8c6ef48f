"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elsi_gpu.h")
LIB = os.path.join(ROOT, "paper_1705_11191_amd", "libelsi_gpu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(elsi_gpu_\w+)\s*\(", text)))


def test_header_declares_core_api():
    names = declared_functions()
    for core in ["elsi_gpu_init", "elsi_gpu_ev", "elsi_gpu_dm", "elsi_gpu_finalize",
                 "elsi_gpu_get_info", "elsi_gpu_workspace_size", "elsi_gpu_set_workspace"]:
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libelsi_gpu.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libelsi_gpu.so not built")
def test_strerror_and_argument_checks_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.elsi_gpu_strerror.restype = ctypes.c_char_p
    assert lib.elsi_gpu_strerror(0) == b"success"
    assert b"positive definite" in lib.elsi_gpu_strerror(1)
    h = ctypes.c_void_p(0)
    lib.elsi_gpu_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
    assert lib.elsi_gpu_init(None, 0, 10, 10, 5.0, None) == -1
    assert lib.elsi_gpu_init(ctypes.byref(h), 3, 10, 10, 5.0, None) == -2
    assert lib.elsi_gpu_init(ctypes.byref(h), 0, 0, 1, 5.0, None) == -3
    assert lib.elsi_gpu_init(ctypes.byref(h), 0, 10, 11, 5.0, None) == -4
    assert lib.elsi_gpu_init(ctypes.byref(h), 0, 10, 10, -1.0, None) == -5
    assert lib.elsi_gpu_init(ctypes.byref(h), 0, 10, 10, 5.0, None) == 0
    lib.elsi_gpu_set_band_width.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.elsi_gpu_set_band_width(h, 12) == -2
    assert lib.elsi_gpu_set_band_width(h, 32) == 0
    # per-size band widths of the batched calls
    IA = ctypes.c_int * 3
    lib.elsi_gpu_set_batch_band_table.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    nmax, bw = IA(512, 1024, 4096), IA(32, 48, 64)
    assert lib.elsi_gpu_set_batch_band_table(None, 3, nmax, bw) == -1
    assert lib.elsi_gpu_set_batch_band_table(h, -1, nmax, bw) == -2
    assert lib.elsi_gpu_set_batch_band_table(h, 17, nmax, bw) == -2
    assert lib.elsi_gpu_set_batch_band_table(h, 3, None, bw) == -3
    assert lib.elsi_gpu_set_batch_band_table(h, 3, IA(512, 512, 4096), bw) == -3
    assert lib.elsi_gpu_set_batch_band_table(h, 3, IA(0, 512, 4096), bw) == -3
    assert lib.elsi_gpu_set_batch_band_table(h, 3, nmax, None) == -4
    assert lib.elsi_gpu_set_batch_band_table(h, 3, nmax, IA(32, 12, 64)) == -4
    assert lib.elsi_gpu_set_batch_band_table(h, 3, nmax, IA(32, 48, 72)) == -4
    assert lib.elsi_gpu_set_batch_band_table(h, 3, nmax, bw) == 0
    assert lib.elsi_gpu_set_batch_band_table(h, 0, None, None) == 0
    lib.elsi_gpu_set_precision.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    assert lib.elsi_gpu_set_precision(None, 1, 1e-10, 4) == -1
    assert lib.elsi_gpu_set_precision(h, 2, 1e-10, 4) == -2
    assert lib.elsi_gpu_set_precision(h, 1, -1.0, 4) == -3
    assert lib.elsi_gpu_set_precision(h, 1, float("nan"), 4) == -3
    assert lib.elsi_gpu_set_precision(h, 1, 1e-10, -1) == -4
    assert lib.elsi_gpu_set_precision(h, 1, 1e-10, 0) == 0
    assert lib.elsi_gpu_set_precision(h, 0, 1e-10, 4) == 0
    # the mixed mode needs n^2 more doubles of workspace than the FP64 mode
    lib.elsi_gpu_workspace_size.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    ws64, wsmx = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.elsi_gpu_workspace_size(h, ctypes.byref(ws64)) == 0
    assert lib.elsi_gpu_set_precision(h, 1, 1e-10, 4) == 0
    assert lib.elsi_gpu_workspace_size(h, ctypes.byref(wsmx)) == 0
    assert wsmx.value >= ws64.value + 10 * 10 * 8
    lib.elsi_gpu_finalize.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    assert lib.elsi_gpu_finalize(ctypes.byref(h)) == 0
    assert h.value is None
    # complex handles take the mixed mode for dm (on the real image): the
    # workspace grows by the refinement's buffers of the 2n image
    assert lib.elsi_gpu_init(ctypes.byref(h), 1, 10, 10, 5.0, None) == 0
    assert lib.elsi_gpu_workspace_size(h, ctypes.byref(ws64)) == 0
    assert lib.elsi_gpu_set_precision(h, 1, 1e-10, 4) == 0
    assert lib.elsi_gpu_workspace_size(h, ctypes.byref(wsmx)) == 0
    assert wsmx.value >= ws64.value + 20 * 20 * 8
    assert lib.elsi_gpu_set_precision(h, 0, 1e-10, 4) == 0
    # the singularity check is for real handles
    lib.elsi_gpu_set_singularity.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
    assert lib.elsi_gpu_set_singularity(h, 1, 1e-5) == -2
    assert lib.elsi_gpu_set_singularity(h, 0, 1e-5) == 0
    assert lib.elsi_gpu_finalize(ctypes.byref(h)) == 0
    # refinement stage entry: argument checks return before any device work
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.elsi_gpu_x_refine.argtypes = [i, i, i, vp, i, vp, i, vp, i, vp, vp, vp, vp, vp, vp, d, i,
                                      ctypes.POINTER(i), vp]
    fake = ctypes.c_void_p(16)
    sw = ctypes.c_int(7)

    def refine(n, k, kw, Ht, ldh, X, ldx, Q=None, ldq=1, dd=None, ee=None, th=fake, rs=fake, tol=1e-10, ms=4,
               swp=None):
        return lib.elsi_gpu_x_refine(n, k, kw, Ht, ldh, X, ldx, Q, ldq, dd, ee, None, th, rs, None, tol, ms, swp,
                                     None)

    assert refine(-1, 0, 0, fake, 1, fake, 1) == -1
    assert refine(4, 5, 0, fake, 4, fake, 4) == -2
    assert refine(4, 2, 3, fake, 4, fake, 4) == -3
    assert refine(4, 2, 2, None, 4, fake, 4) == -4
    assert refine(4, 2, 2, fake, 3, fake, 4) == -4
    assert refine(4, 2, 2, fake, 4, fake, 3) == -6
    assert refine(4, 2, 2, fake, 4, fake, 4, Q=fake, ldq=3, dd=fake, ee=fake) == -9
    assert refine(4, 2, 2, fake, 4, fake, 4, Q=fake, ldq=4, dd=None, ee=fake) == -10
    assert refine(4, 2, 2, fake, 4, fake, 4, Q=fake, ldq=4, dd=fake, ee=None) == -11
    assert refine(4, 2, 2, fake, 4, fake, 4, th=None) == -13
    assert refine(4, 2, 2, fake, 4, fake, 4, rs=None) == -14
    assert refine(4, 2, 2, fake, 4, fake, 4, tol=-1.0) == -16
    assert refine(4, 2, 2, fake, 4, fake, 4, ms=-1) == -17
    assert refine(0, 0, 0, None, 1, None, 1, th=None, rs=None, swp=ctypes.byref(sw)) == 0
    assert sw.value == 0
    # back-transformation stage entry
    lib.elsi_gpu_x_backtransform.argtypes = [i, i, vp, i, vp, vp, vp, i, i, i, i, vp]
    assert lib.elsi_gpu_x_backtransform(0, 8, fake, 1, fake, fake, fake, 1, 1, 0, 0, None) == -1
    assert lib.elsi_gpu_x_backtransform(8, 65, fake, 8, fake, fake, fake, 8, 1, 0, 0, None) == -2
    assert lib.elsi_gpu_x_backtransform(8, 8, fake, 8, fake, fake, fake, 8, 1, 2, 0, None) == -10
    assert lib.elsi_gpu_x_backtransform(8, 8, fake, 8, fake, fake, fake, 8, 1, 0, 64, None) == -11
    # the allocation-free Cholesky rejects sizes beyond its fixed scratch on
    # the host, before any GPU call
    lib.elsi_gpu_x_cholesky_noalloc.argtypes = [i, vp, i, ctypes.POINTER(i), vp]
    fc = ctypes.c_int(3)
    assert lib.elsi_gpu_x_cholesky_noalloc(16385, fake, 16385, ctypes.byref(fc), None) == -1
    assert lib.elsi_gpu_x_cholesky_noalloc(-1, fake, 1, ctypes.byref(fc), None) == -1
    assert lib.elsi_gpu_x_cholesky_noalloc(0, None, 1, ctypes.byref(fc), None) == 0 and fc.value == 0


def test_product_path_does_not_import_oracle():
    # the GPU package and binding must not reach into the CPU oracle
    pkg = os.path.join(ROOT, "paper_1705_11191_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "elsi_oracle" not in src and "liborc" not in src, f
