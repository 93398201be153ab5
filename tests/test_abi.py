"""The C-ABI library loads and exports every entry point declared in include/hbj.h (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2209_10886_amd", "libhbj.so")
HEADER = os.path.join(ROOT, "include", "hbj.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hbj_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("hbj_setup", "hbj_factor", "hbj_apply_preconditioner", "hbj_apply_operator", "hbj_solve",
              "hbj_gradient", "hbj_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_2209_10886_amd as hbj

    assert set(declared()) <= set(hbj.EXPORTED)


def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.hbj_strerror.restype = ctypes.c_char_p
    assert lib.hbj_strerror(0) == b"ok"
    assert b"singular" in lib.hbj_strerror(1)
    assert b"converge" in lib.hbj_strerror(2)


def test_setup_rejects_bad_sizes_before_touching_the_gpu():
    """Size validation happens on the host before any HIP call."""
    import paper_2209_10886_amd as hbj

    lib = hbj._lib
    out = ctypes.c_void_p()
    for (nx, ny, n1, n2) in [(10, 10, 3, 2), (4, 4, 4, 1), (0, 8, 1, 1)]:
        p = hbj.Problem(nx, ny, 0.0, 10.0, n1, n2, 0, 2, 0, 0, 0, 0, 0)
        code = lib.hbj_setup(ctypes.byref(p), ctypes.c_void_p(16), None, ctypes.byref(out))
        assert code == hbj.EINVAL
    p = hbj.Problem(16, 16, 0.0, 10.0, 2, 2, 7, 2, 0, 0, 0, 0, 0)  # bad precision
    assert lib.hbj_setup(ctypes.byref(p), ctypes.c_void_p(16), None, ctypes.byref(out)) == hbj.EINVAL


def test_setup_rejects_bad_options_on_the_host():
    import paper_2209_10886_amd as hbj

    lib = hbj._lib
    out = ctypes.c_void_p()
    bad = [dict(precond=5), dict(bj_width=-1), dict(bj_combine=2), dict(bj_compose=3), dict(operator_form=2),
           dict(sweep_exec=2), dict(sweep_exec=-1), dict(transmission=3), dict(transmission=-1)]
    for kw in bad:
        args = dict(precision=0, precond=2, bj_width=0, bj_combine=0, bj_compose=0, operator_form=0, sweep_exec=0,
                    transmission=0)
        args.update(kw)
        p = hbj.Problem(16, 16, 0.0, 10.0, 2, 2, args["precision"], args["precond"], args["bj_width"],
                        args["bj_combine"], args["bj_compose"], args["operator_form"], args["sweep_exec"],
                        args["transmission"])
        assert lib.hbj_setup(ctypes.byref(p), ctypes.c_void_p(16), None, ctypes.byref(out)) == hbj.EINVAL
