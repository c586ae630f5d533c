"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/hsb.h, and rejects invalid arguments before device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_08361_amd import hsb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hsb.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hsb_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_entry_points():
    assert set(_declared()) == set(hsb.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = hsb.load_library()
    for name in _declared():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


@pytest.mark.parametrize("struct", ["hsb_run_args", "hsb_job", "hsb_batch_args"])
def test_struct_layout_matches_header(tmp_path, struct):
    """ctypes layout of each argument struct equals what a C compiler makes of the header."""
    cls = getattr(hsb, struct)
    fields = [f[0] for f in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"hsb.h\"\nint main(void){\n"
                   + 'printf("%%zu\\n", sizeof(%s));\n' % struct
                   + "".join('printf("%%zu\\n", offsetof(%s, %s));\n' % (struct, f) for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cls)
    for f, off in zip(fields, vals[1:]):
        assert getattr(cls, f).offset == off, f


def test_constants_match_header(tmp_path):
    """Every HSB_* enumerator and return code of the header has the binding's value."""
    text = open(os.path.join(ROOT, "include", "hsb.h")).read()
    names = sorted(set(re.findall(r"\b(HSB_(?:OK|E[A-Z]+|OPT_[A-Z_]+|PREC_[A-Z0-9_]+|PLAN_[A-Z0-9]+|"
                                  r"DSB|BSB))\b", text)))
    names = [n for n in names if hasattr(hsb, n)]
    assert len(names) >= 20
    src = tmp_path / "consts.c"
    src.write_text("#include <stdio.h>\n#include \"hsb.h\"\nint main(void){\n"
                   + "".join('printf("%%d\\n", (int)%s);\n' % n for n in names) + "return 0;}\n")
    exe = tmp_path / "consts"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    for n, v in zip(names, vals):
        assert getattr(hsb, n) == v, n


def _create_rc(J, N=None):
    L = hsb.load_library()
    J = np.ascontiguousarray(J, dtype=np.float32)
    h = ctypes.c_void_p()
    rc = L.hsb_create(J.ctypes.data, J.shape[0] if N is None else N, ctypes.byref(h))
    return rc, h, hsb.hsb_last_error()


@pytest.mark.parametrize("bad,msg", [
    (np.array([[0, 1], [2, 0]]), "symmetric"),
    (np.array([[1, 0], [0, 0]]), "diagonal"),
    (np.array([[0, np.nan], [np.nan, 0]]), "finite"),
    (np.array([[0, np.inf], [np.inf, 0]]), "finite"),
])
def test_create_rejects_invalid_J(bad, msg):
    rc, h, err = _create_rc(bad)
    assert rc == hsb.HSB_EINVAL and msg in err and not h.value


def test_create_rejects_bad_sizes_and_nulls():
    rc, h, err = _create_rc(np.zeros((2, 2)), N=0)
    assert rc == hsb.HSB_EINVAL
    L = hsb.load_library()
    h = ctypes.c_void_p()
    assert L.hsb_create(None, 4, ctypes.byref(h)) == hsb.HSB_EINVAL
    J = np.zeros((2, 2), dtype=np.float32)
    assert L.hsb_create(J.ctypes.data, 2, None) == hsb.HSB_EINVAL


def test_calls_on_null_context_are_rejected():
    L = hsb.load_library()
    assert L.hsb_run(None, 0, 1.0, 0.1, 1.0, 0.0, 10, 4, 0, None, None) == hsb.HSB_EINVAL
    assert L.hsb_run_ex(None, None) == hsb.HSB_EINVAL
    assert L.hsb_run_ex_noalloc(None, None) == hsb.HSB_EINVAL
    assert L.hsb_cancel(None) == hsb.HSB_EINVAL
    assert L.hsb_set_option(None, 0, 0.1) == hsb.HSB_EINVAL
    a = hsb.hsb_batch_args()
    a.struct_size = ctypes.sizeof(a)
    assert L.hsb_run_batch(None, 1, None, 0, ctypes.byref(a)) == hsb.HSB_EINVAL
    n = ctypes.c_int(-7)
    assert L.hsb_num_samples(None, 0, 10, ctypes.byref(n)) == hsb.HSB_EINVAL
    assert n.value == -7
    L.hsb_destroy(None)  # ignored


def test_noalloc_scratch_size_matches_header():
    text = open(os.path.join(ROOT, "include", "hsb.h")).read()
    m = re.search(r"#define HSB_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == hsb.HSB_NOALLOC_SCRATCH_BYTES


def test_valid_J_without_gpu_is_a_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h, err = _create_rc(np.array([[0, 1], [1, 0]]))
    assert rc == hsb.HSB_EDEVICE and not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libhsb.so the binding raises; there is no other execution path."""
    monkeypatch.setattr(hsb, "LIB_PATH", str(tmp_path / "absent" / "libhsb.so"))
    monkeypatch.setattr(hsb, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        hsb.load_library()
    with pytest.raises(RuntimeError, match="not built"):
        hsb.Context(np.zeros((4, 4), dtype=np.float32))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    (before touching any device)."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
