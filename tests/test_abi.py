"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/bk.h declares, sizes its workspaces, and rejects bad
arguments with BK_EINVAL before launching anything."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1504_05477_amd as bk
from paper_1504_05477_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "bk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bk_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return bk.load()


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", bk.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    declared = _declared()
    assert len(declared) >= 18
    missing = [s for s in declared if s not in syms]
    assert not missing, missing
    # and the binding knows every one of them
    assert set(declared) <= set(L.EXPORTS)


def test_status_strings(lib):
    assert lib.bk_status_string(0) == b"ok"
    assert b"rank" in lib.bk_status_string(6)
    assert lib.bk_version().startswith(b"bk ")


def test_struct_layouts():
    assert C.sizeof(L.Options) == 112
    assert L.Options.residuals.offset == 72
    assert L.Options.at_scales.offset == 96
    assert L.Info.workspace_bytes.offset == 112
    assert C.sizeof(L.Metrics) == 56


def test_struct_layouts_match_the_c_header(tmp_path):
    # every field of the ctypes mirrors sits where a C compiler puts it
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bk.h"', "int main(void) {"]
    for cname, py in (("bk_options", L.Options), ("bk_info", L.Info), ("bk_metrics", L.Metrics)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "lay.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run([cc, f"-I{inc}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, py in (("bk_options", L.Options), ("bk_info", L.Info), ("bk_metrics", L.Metrics)):
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def _opt():
    o = L.Options()
    o.struct_size = C.sizeof(L.Options)
    return o


def test_workspace_sizes(lib):
    o = _opt()
    small = lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o))
    assert small > 2000 * 90 * 8
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F32, C.byref(o)) < small
    assert lib.bk_svd_dense_workspace(2000, 1000, 0, 8, L.F64, C.byref(o)) == 0
    assert lib.bk_svd_dense_workspace(100, 50, 10, 5, L.F64, C.byref(o)) == 0  # m > d
    assert lib.bk_svd_csr_workspace(11000, 130000, 1_500_000, 20, 10, C.byref(o)) > 0
    assert lib.bk_svd_csr_workspace(10, 10, 2**31, 2, 1, C.byref(o)) == 0
    assert lib.bk_eigh_psd_workspace(90) > 90 * 90 * 8


def test_block_size_and_method_rules(lib):
    """Oversampling (block width p >= k) and Simultaneous Iteration are
    validated at the boundary: the workspace query returns 0 on a bad p."""
    base = lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(_opt()))
    o = _opt()
    o.block_size = 12
    wide = lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o))
    assert wide > base                                    # 9 blocks of 12 columns
    o.block_size = 9                                      # p < k
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o)) == 0
    o.block_size = 200                                    # (q+1) p > min(n, d)
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o)) == 0
    o.method = 1                                          # Algorithm 1: p <= min(n, d)
    si = lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o))
    assert si > 0
    o.save_for_backward = 1                               # no adjoint for Algorithm 1
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o)) == 0
    o = _opt()
    o.method = 2                                          # block Lanczos: T's blocks kept
    bl = lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o))
    assert bl > base
    o.save_for_backward = 1                               # no adjoint for it either
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o)) == 0
    o = _opt()
    o.block_size = 30
    assert lib.bk_svd_csr_workspace(11000, 130000, 1_500_000, 20, 10, C.byref(o)) > \
        lib.bk_svd_csr_workspace(11000, 130000, 1_500_000, 20, 10, C.byref(_opt()))


@pytest.mark.parametrize("n,d,k,q", [(100, 50, 0, 1), (100, 50, 51, 0), (100, 50, 5, -1),
                                     (100, 50, 10, 5), (0, 50, 1, 0)])
def test_dense_rejects_bad_shapes(lib, n, d, k, q):
    st = lib.bk_svd_dense(C.c_void_p(16), 50, L.F32, None, None, 0, n, d, k, q, 0, None,
                          C.c_void_p(16), 10, C.c_void_p(16), None, None, 0, None)
    assert st == L.EINVAL


def test_dense_rejects_bad_pointers_and_strides(lib):
    args = dict(n=100, d=50, k=5, q=1)
    # null A
    assert lib.bk_svd_dense(None, 50, L.F32, None, None, 0, 100, 50, 5, 1, 0, None,
                            C.c_void_p(16), 5, C.c_void_p(16), None, None, 0, None) == L.EINVAL
    # lda < d
    assert lib.bk_svd_dense(C.c_void_p(16), 49, L.F32, None, None, 0, 100, 50, 5, 1, 0, None,
                            C.c_void_p(16), 5, C.c_void_p(16), None, None, 0, None) == L.EINVAL
    # FP8 without scales
    assert lib.bk_svd_dense(C.c_void_p(16), 50, L.FP8_E4M3, None, None, 0, 100, 50, 5, 1, 0,
                            None, C.c_void_p(16), 5, C.c_void_p(16), None, None, 0,
                            None) == L.EINVAL
    # refine requested without a master copy
    o = _opt()
    o.refine = 1
    assert lib.bk_svd_dense(C.c_void_p(16), 50, L.BF16, None, None, 0, 100, 50, 5, 1, 0,
                            C.byref(o), C.c_void_p(16), 5, C.c_void_p(16), None, None, 0,
                            None) == L.EINVAL
    # unknown dtype
    assert lib.bk_svd_dense(C.c_void_p(16), 50, 7, None, None, 0, 100, 50, 5, 1, 0, None,
                            C.c_void_p(16), 5, C.c_void_p(16), None, None, 0, None) == L.EINVAL
    del args


def test_csr_and_helpers_reject_bad_arguments(lib):
    assert lib.bk_svd_csr(None, None, None, None, None, None, 10, 10, 5, 2, 1, 0, None,
                          C.c_void_p(16), 2, C.c_void_p(16), None, None, 0, None) == L.EINVAL
    # half a transpose given
    assert lib.bk_svd_csr(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16),
                          None, None, 10, 10, 5, 2, 1, 0, None, C.c_void_p(16), 2,
                          C.c_void_p(16), None, None, 0, None) == L.EINVAL
    assert lib.bk_gaussian(0, 4, 4, 3, L.F32, C.c_void_p(16), None) == L.EINVAL
    assert lib.bk_gaussian(0, 4, 4, 4, L.BF16, C.c_void_p(16), None) == L.EINVAL
    assert lib.bk_quantize_dense(C.c_void_p(16), 4, 4, 4, L.FP8_E4M3, C.c_void_p(16), None,
                                 None) == L.EINVAL
    assert lib.bk_eigh_psd(None, 4, 4, None, None, 4, 0, 0.0, None, None, 0, None) == L.EINVAL
    assert lib.bk_dense_product(0, C.c_void_p(16), 3, L.F32, None, 4, 4, C.c_void_p(16), 2, 2,
                                C.c_void_p(16), 2, None, 0, None) == L.EINVAL


def test_error_metrics_argument_rules(lib):
    """The error-measure calls validate shapes and types before any GPU work."""
    assert lib.bk_error_metrics_dense_workspace(600, 400, 8, 4, L.F64) > 600 * 8 * 8
    assert lib.bk_error_metrics_dense_workspace(600, 400, 8, 4, L.BF16) == 0
    assert lib.bk_error_metrics_dense_workspace(600, 400, 8, 60, L.F32) == 0  # (q+1) k > d
    assert lib.bk_error_metrics_csr_workspace(11000, 130000, 1_500_000, 20, 4) > 0
    assert lib.bk_error_metrics_csr_workspace(10, 10, 2**31, 2, 1) == 0
    P = C.c_void_p(16)
    # unsupported A type, ldz < k, lda < d, null Z
    assert lib.bk_error_metrics_dense(P, 400, L.BF16, 600, 400, P, 8, 8, 4, 0, None, 0, None,
                                      None, None, 0, None) == L.EINVAL
    assert lib.bk_error_metrics_dense(P, 400, L.F32, 600, 400, P, 7, 8, 4, 0, None, 0, None,
                                      None, None, 0, None) == L.EINVAL
    assert lib.bk_error_metrics_dense(P, 399, L.F32, 600, 400, P, 8, 8, 4, 0, None, 0, None,
                                      None, None, 0, None) == L.EINVAL
    assert lib.bk_error_metrics_dense(P, 400, L.F32, 600, 400, None, 8, 8, 4, 0, None, 0, None,
                                      None, None, 0, None) == L.EINVAL
    # CSR: null row_ptr, half a transpose, q_spec too deep
    assert lib.bk_error_metrics_csr(None, P, P, None, None, None, 10, 10, 5, 0, P, 2, 2, 1, 0,
                                    None, 0, None, None, None, 0, None) == L.EINVAL
    assert lib.bk_error_metrics_csr(P, P, P, P, None, None, 10, 10, 5, 0, P, 2, 2, 1, 0, None,
                                    0, None, None, None, 0, None) == L.EINVAL
    assert lib.bk_error_metrics_csr(P, P, P, None, None, None, 10, 10, 5, 0, P, 2, 2, 5, 0,
                                    None, 0, None, None, None, 0, None) == L.EINVAL


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        L.load(str(tmp_path / "libbk.so"))


def test_binding_rejects_host_tensors_and_type_mismatch():
    """The Python binding checks placement and types before any library call."""
    torch = pytest.importorskip("torch")
    import paper_1504_05477_amd as bk
    A = torch.zeros(8, 6, dtype=torch.float64)
    Z = torch.zeros(8, 2, dtype=torch.float64)
    with pytest.raises(ValueError):
        bk.error_metrics_dense(A, Z)                       # host tensors
    with pytest.raises(ValueError):
        bk.svd_dense(A, 2, 1)
    rp = torch.zeros(9, dtype=torch.int32)
    with pytest.raises(ValueError):
        bk.error_metrics_csr(rp, rp[:0], torch.zeros(0), 8, 6, Z.float())


def test_too_small_workspace_gives_enomem(lib):
    """A caller-given workspace one byte short of the queried size is
    rejected with BK_ENOMEM before anything is enqueued (no GPU needed: the
    pointers are never dereferenced)."""
    P = C.c_void_p(4096)
    o = _opt()
    for code in (L.F64, L.F32):
        need = lib.bk_svd_dense_workspace(600, 400, 8, 4, code, C.byref(o))
        assert need > 0
        st = lib.bk_svd_dense(P, 400, code, None, None, 0, 600, 400, 8, 4, 0, C.byref(o), P, 8,
                              P, None, P, need - 1, None)
        assert st == L.ENOMEM
    # the backward, given a forward workspace of the right size
    o.save_for_backward = 1
    fwd = lib.bk_svd_dense_workspace(600, 400, 8, 4, L.F32, C.byref(o))
    need = lib.bk_svd_dense_backward_workspace(600, 400, 8, 4, L.F32)
    assert need > 0
    st = lib.bk_svd_dense_backward(P, 400, L.F32, 600, 400, 8, 4, P, 8, P, P, P, P, 400, P,
                                   fwd, P, need - 1, None)
    assert st == L.ENOMEM
    # CSR (transpose built inside, and given)
    o = _opt()
    need = lib.bk_svd_csr_workspace(500, 3000, 9000, 6, 3, C.byref(o))
    assert need > 0
    st = lib.bk_svd_csr(P, P, P, None, None, None, 500, 3000, 9000, 6, 3, 0, C.byref(o), P, 6,
                        P, None, P, need - 1, None)
    assert st == L.ENOMEM
    st = lib.bk_svd_csr(P, P, P, P, P, P, 500, 3000, 9000, 6, 3, 0, C.byref(o), P, 6, P, None,
                        P, 4096, None)
    assert st == L.ENOMEM
    # error measures and the block product
    need = lib.bk_error_metrics_dense_workspace(600, 400, 8, 4, L.F32)
    assert lib.bk_error_metrics_dense(P, 400, L.F32, 600, 400, P, 8, 8, 4, 0, None, 0, None,
                                      None, P, need - 1, None) == L.ENOMEM
    need = lib.bk_dense_product_workspace(1, 600, 400, 8, L.F32)
    if need > 0:
        assert lib.bk_dense_product(1, P, 400, L.F32, None, 600, 400, P, 8, 8, P, 8, P,
                                    need - 1, None) == L.ENOMEM


def test_noalloc_size_limit_and_rules(lib):
    """The allocation-free solve rejects a problem whose workspace exceeds
    its static scratch (BK_ENOMEM) and a save_for_backward request
    (BK_EINVAL) before touching the device (no GPU needed)."""
    P = C.c_void_p(4096)
    limit = 64 << 20
    o = _opt()
    assert lib.bk_svd_dense_workspace(2000, 1000, 10, 8, L.F64, C.byref(o)) <= limit
    big = lib.bk_svd_dense_workspace(8192, 4096, 32, 10, L.F32, C.byref(o))
    assert big > limit
    assert lib.bk_svd_dense_noalloc(P, 4096, L.F32, None, None, 0, 8192, 4096, 32, 10, 0,
                                    C.byref(o), P, 32, P, None, None) == L.ENOMEM
    o.save_for_backward = 1
    assert lib.bk_svd_dense_noalloc(P, 1000, L.F64, None, None, 0, 2000, 1000, 10, 8, 0,
                                    C.byref(o), P, 10, P, None, None) == L.EINVAL
    o = _opt()
    assert lib.bk_svd_dense_noalloc(None, 1000, L.F64, None, None, 0, 2000, 1000, 10, 8, 0,
                                    C.byref(o), P, 10, P, None, None) == L.EINVAL
    assert lib.bk_svd_dense_noalloc(P, 1000, L.F64, None, None, 0, 2000, 1000, 0, 8, 0,
                                    C.byref(o), P, 10, P, None, None) == L.EINVAL
