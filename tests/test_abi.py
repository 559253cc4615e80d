"""Host-side checks of the C ABI (no GPU work): the library loads, exports every
function include/altgdmin.h declares, the ctypes structs of the binding have the
C layout, and the host-only entry points validate their arguments as documented.
"""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "altgdmin.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(altgdmin_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_functions(lib):
    declared = set(_declared_functions())
    assert declared == set(lib.EXPORTED), (declared ^ set(lib.EXPORTED))


def test_library_exports_every_declared_symbol(lib):
    so = lib.load()
    missing = [f for f in _declared_functions() if not hasattr(so, f)]
    assert not missing, missing


_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "altgdmin.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("altgdmin_problem sizeof %zu\n", sizeof(altgdmin_problem));
  printf("altgdmin_params sizeof %zu\n", sizeof(altgdmin_params));
  printf("altgdmin_report sizeof %zu\n", sizeof(altgdmin_report));
  %FIELDS%
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_struct_layouts_match_c(lib, tmp_path):
    structs = {"altgdmin_problem": lib.Problem, "altgdmin_params": lib.Params, "altgdmin_report": lib.Report}
    fields = "\n  ".join(f"F({c}, {f})" for c, py in structs.items() for f, _ in py._fields_)
    src = tmp_path / "probe.c"
    src.write_text(_PROBE.replace("%FIELDS%", fields))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for c, py in structs.items():
        assert got[(c, "sizeof")] == ctypes.sizeof(py), c
        for f, _ in py._fields_:
            assert got[(c, f)] == getattr(py, f).offset, (c, f)


def _problem(lib, **kw):
    """A problem whose device pointers are placeholders: only validated, never dereferenced."""
    p = lib.Problem()
    p.n, p.q, p.m, p.r, p.rho = 1000, 1000, 400, 10, 50
    p.a_format = lib.ALTGDMIN_A_F32
    p.A, p.Y = 1 << 20, 1 << 24
    p.lda, p.a_stride_k, p.ldy = 400, 400 * 1000, 400
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ws(lib, p, par=None):
    so = lib.load()
    par = par or lib.default_params()
    b = ctypes.c_size_t(0)
    rc = so.altgdmin_workspace_bytes(ctypes.byref(p), ctypes.byref(par), ctypes.byref(b))
    return rc, b.value, so.altgdmin_last_error().decode()


def test_default_params_are_the_papers(lib):
    par = lib.default_params()
    assert (par.tau0, par.tau, par.t_max) == (10, 3, 200)
    assert par.eta_c == pytest.approx(0.14)
    assert par.tol_resid == 0.0 and par.flags == 0


@pytest.mark.parametrize("n, m, r", [(17688, 1024, 16), (17104, 400, 10), (19692, 64, 4), (16384, 400, 10)])
def test_large_n_is_accepted_up_to_the_lds_of_a_cu(lib, n, m, r):
    """g, the step and the support bitmap of a column are n-long LDS arrays; up to the
    CU's 160 KiB (one column workgroup per CU) every n up to these is built, which
    includes 128 x 128 frames (n = 16384) at the benchmark's m and r."""
    lda = (m + 7) // 8 * 8
    rc, b, _ = _ws(lib, _problem(lib, n=n, m=m, r=r, lda=lda, ldy=m, a_stride_k=lda * n))
    assert rc == 0 and b > 0
    rc, _, _ = _ws(lib, _problem(lib, n=n + 1, m=m, r=r, lda=lda, ldy=m, a_stride_k=lda * (n + 1)))
    assert rc == (-5 if n != 16384 else 0)


def test_workspace_bytes_accepts_the_benchmark_problem(lib):
    rc, b, _ = _ws(lib, _problem(lib))
    assert rc == 0 and b > 0
    rc2, b2, _ = _ws(lib, _problem(lib, q=2000))
    assert rc2 == 0 and b2 > b          # per-column state grows with q
    assert b % 256 == 0


@pytest.mark.parametrize("kw, code", [
    (dict(r=17), -5),                   # no instantiation above r = 16
    (dict(n=17689, m=1024, r=16, lda=1024, ldy=1024, a_stride_k=1024 * 17689), -5),   # 160 KiB LDS of a column workgroup
    (dict(m=1025, lda=1028, a_stride_k=1028 * 1000, ldy=1025), -5),
    (dict(r=-1), -1),                   # r = 0 is the automatic rank; negative is invalid
    (dict(q=0), -1),                    # empty problem
    (dict(n=0), -1),
    (dict(m=0, lda=4, ldy=4, a_stride_k=4000), -1),
    (dict(r=12, m=10, lda=12, ldy=12, a_stride_k=12000), -1),   # r > m
    (dict(rho=1001), -1),
    (dict(rho=-1), -1),
    (dict(lda=402), -1),                # not a multiple of 4
    (dict(lda=396), -1),                # lda < m
    (dict(a_stride_k=400 * 999), -1),   # A_k overlap
    (dict(ldy=399), -1),
    (dict(A=None), -1),
    (dict(Y=None), -1),
    (dict(A=(1 << 20) + 4), -1),        # base not 16-byte aligned
    (dict(a_format=7), -1),
    (dict(a_format=1), -1),             # BF16X2 without the lo plane
    (dict(a_format=2), -1),             # PHILOX without the normal table
])
def test_workspace_bytes_rejects_invalid_problems(lib, kw, code):
    rc, _, msg = _ws(lib, _problem(lib, **kw))
    assert rc == code
    assert msg


def test_workspace_bytes_rejects_invalid_params(lib):
    for field, value in [("tau", -1), ("t_max", -1), ("poll_every", 0), ("eta_c", -0.1), ("bf16_hi_max", -2), ("flags", 4)]:
        par = lib.default_params(**{field: value})
        rc, _, _ = _ws(lib, _problem(lib), par)
        assert rc == -1, field


def test_philox_problem_needs_no_A(lib):
    p = _problem(lib, a_format=2, A=None, lda=0, a_stride_k=0)
    p.normal_table = 1 << 22
    rc, b, _ = _ws(lib, p)
    assert rc == 0 and b > 0


def test_strerror_covers_every_code(lib):
    so = lib.load()
    texts = {c: so.altgdmin_strerror(c).decode() for c in (0, 1, -1, -2, -3, -4, -5)}
    assert all(texts.values())
    assert len(set(texts.values())) == len(texts)


def test_op_scratch_bytes_is_host_only(lib):
    so = lib.load()
    b = ctypes.c_size_t(0)
    assert so.altgdmin_op_scratch_bytes(1000, 1000, 10, ctypes.byref(b)) == 0
    assert b.value >= 4 * 1000 * 10
    assert so.altgdmin_op_scratch_bytes(0, 1000, 10, ctypes.byref(b)) < 0


def _fourier_problem(lib, **kw):
    p = lib.Problem()
    p.n, p.q, p.m, p.r, p.rho = 96 * 96, 64, 1536, 6, 184
    p.n1 = p.n2 = 96
    p.a_format = lib.ALTGDMIN_A_PFOURIER
    p.fourier_mask, p.Y, p.ldy = 1 << 20, 1 << 24, 1536
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_fourier_workspace_and_limits(lib):
    rc, b, _ = _ws(lib, _fourier_problem(lib))
    assert rc == 0 and b >= 8 * 64 * 96 * 96     # holds the q x n complex back-projections
    for kw, code in [(dict(n1=64, n2=144), -5), (dict(n2=95), -1), (dict(r=9), -5), (dict(rho=257), -5),
                     (dict(m=2049, ldy=2049), -5), (dict(fourier_mask=None), -1), (dict(ldy=100), -1),
                     (dict(m=9217), -1)]:
        rc, _, msg = _ws(lib, _fourier_problem(lib, **kw))
        assert rc == code, (kw, msg)


def test_null_stream_is_rejected_before_any_gpu_work(lib):
    """The library never enqueues on the null stream: every entry point that takes a
    stream returns EINVAL for NULL (checked here with placeholder device pointers,
    which are validated but never dereferenced)."""
    so = lib.load()
    p = _problem(lib)
    par = lib.default_params()
    h = ctypes.c_void_p()
    assert so.altgdmin_init(ctypes.byref(p), ctypes.byref(par), 1 << 30, 1 << 34, None, ctypes.byref(h)) == -1
    assert "stream" in so.altgdmin_last_error().decode()
    assert so.altgdmin_op_select(1 << 20, 100, 4, 100, 5, 1 << 21, 1 << 22, None, None) == -1
    assert so.altgdmin_op_au(ctypes.byref(p), 1 << 20, 1 << 21, 1 << 22, None, None) == -1
    assert so.altgdmin_op_iht(ctypes.byref(p), 0, None, None, 1, 0, 1 << 20, 1 << 21, None, None, None, None) == -1
    assert so.altgdmin_op_grad(1 << 20, 1 << 21, 100, 100, 2, 1 << 22, 1 << 23, 1 << 20, None) == -1


def test_state_entry_points_validate_arguments(lib):
    so = lib.load()
    b = ctypes.c_size_t(0)
    assert so.altgdmin_state_bytes(None, ctypes.byref(b)) == -1
    assert so.altgdmin_get_state(None, 1 << 20, 1 << 20, 1 << 12) == -1
    assert so.altgdmin_set_state(None, 1 << 20, 1 << 20, 1 << 12) == -1


def test_noalloc_entry_point_checks_sizes_and_stream_on_the_host(lib):
    """Sizes whose scratch exceeds the static array are refused before any GPU call."""
    so = lib.load()
    fake = 1 << 30
    b = ctypes.c_size_t(0)
    assert so.altgdmin_op_scratch_bytes(300000, 1000, 16, ctypes.byref(b)) == 0
    assert b.value > 16 << 20
    assert so.altgdmin_op_subspace_noalloc(fake, 300000, 1000, 16, None, 5, 1e-7, fake, None, 1 << 12) == -2
    assert "static" in so.altgdmin_last_error().decode()
    assert so.altgdmin_op_subspace_noalloc(fake, 1000, 1000, 10, None, 5, 1e-7, fake, None, None) == -1
    assert so.altgdmin_op_subspace_noalloc(fake, 1000, 1000, 17, None, 5, 1e-7, fake, None, 1 << 12) == -1


def test_automatic_rank_problems(lib):
    """r = 0 asks for the automatic rank: the workspace is laid out for the largest rank
    the rule may pick (plus, in the Fourier form, the real embedding of L_0); K > 88 (44
    in the Fourier form) is not built; bad energies are refused."""
    rc0, b0, _ = _ws(lib, _problem(lib, r=0))
    rc16, b16, _ = _ws(lib, _problem(lib, r=16))
    assert rc0 == 0 and rc16 == 0 and b0 > b16 > 0      # r_cap = 16 plus the estimate's scratch
    rc, _, msg = _ws(lib, _problem(lib, r=0, n=2000, q=2000, m=1000, lda=1000, ldy=1000,
                                   a_stride_k=1000 * 2000))
    assert rc == -5 and "automatic rank" in msg      # K = 100 > 88
    rc0, b0, _ = _ws(lib, _fourier_problem(lib, r=0))
    rc6, b6, _ = _ws(lib, _fourier_problem(lib, r=6))
    assert rc0 == 0 and rc6 == 0 and b0 >= b6 + 4 * 4 * 64 * 96 * 96   # K = 6 = r_cap, plus the 2q x 2n embedding
    # 96 x 96 frames, q = 450, m = 900: K = min(n, q, m) / 10 = 45, so 2K = 90 > 88
    rc, _, msg = _ws(lib, _fourier_problem(lib, r=0, q=450, m=900, ldy=900))
    assert rc == -5 and "automatic rank" in msg
    rc, _, _ = _ws(lib, _fourier_problem(lib, r=0, q=440, m=900, ldy=900))   # K = 44
    assert rc == 0
    rc, _, _ = _ws(lib, _problem(lib, r=0), lib.default_params(rank_energy=1.5))
    assert rc == -1
    so = lib.load()
    b = ctypes.c_size_t(0)
    assert so.altgdmin_op_rank_scratch_bytes(1000, 1000, 400, ctypes.byref(b)) == 0 and b.value > 0
    assert so.altgdmin_op_rank_scratch_bytes(2000, 2000, 1000, ctypes.byref(b)) == -5


def test_every_binding_call_that_takes_a_stream_is_ordered_on_a_created_stream():
    """Each binding function with a `stream=` argument is wrapped exactly once by the
    decorator that moves calls off torch's null stream (the library refuses NULL)."""
    src = open(os.path.join(ROOT, "paper_2311_03824_amd", "altgdmin.py")).read().split("\n")
    checked = 0
    for i, line in enumerate(src):
        if not line.startswith("def altgdmin_"):
            continue
        j, sig = i, line
        while not sig.rstrip().endswith(":"):
            j += 1
            sig += src[j]
        takes_stream = "stream=None" in sig
        wrapped = src[i - 1].strip() == "@_on_stream"
        twice = src[i - 2].strip() == "@_on_stream"
        assert takes_stream == wrapped and not twice, line
        checked += takes_stream
    assert checked >= 20


def test_binding_error_codes_match_the_header():
    import re
    from paper_2311_03824_amd import altgdmin as lib
    hdr = open(os.path.join(ROOT, "include", "altgdmin.h")).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"(ALTGDMIN_E[A-Z]+|ALTGDMIN_OK)\s*=\s*(-?\d+)", hdr))
    assert len(codes) == 7
    for name, value in codes.items():
        assert getattr(lib, name) == value, name
