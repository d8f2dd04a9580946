"""The C ABI library (CPU-only checks: it loads, exports every declared call,
and validates shapes without touching a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgn.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1205_2584_amd import dgn
    if not os.path.exists(dgn.LIB_PATH):
        from paper_1205_2584_amd import build
        build.build()
    return dgn.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(\w+)\s*\(", text, flags=re.M)) - {"if"})


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dgn_create", "dgn_destroy", "dgn_last_error", "dgn_workspace_size", "dgn_mttkrp",
              "dgn_step", "cp_fit", "dgn_opts_default"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1205_2584_amd import dgn
    assert set(dgn.EXPORTS) == set(declared_functions())


def test_opts_defaults(lib):
    from paper_1205_2584_amd import dgn
    o = dgn.dgn_opts()
    lib.dgn_opts_default(ctypes.byref(o))
    assert o.normalize == 0 and o.tau == 1e-3 and o.resid_switch == 1e-3 and o.poll_every == 8


@pytest.mark.parametrize("dims,R,ok", [
    ((20, 20, 20), 3, True), ((500, 500, 500), 30, True), ((3, 4, 5, 6, 7), 3, True),
    ((4, 4), 2, False), ((4, 4, 4), 0, False), ((4, 4, 4), 65, False), ((4, 0, 4), 2, False),
    ((2,) * 9, 2, False),
])
def test_workspace_size_validates(lib, dims, R, ok):
    from paper_1205_2584_amd import dgn
    d = dgn.dgn_tensor()
    d.order = len(dims)
    for k, v in enumerate(dims[:8]):
        d.dims[k] = v
    d.dtype = dgn.F32
    d.data = 1
    n = ctypes.c_size_t()
    st = lib.dgn_workspace_size(ctypes.byref(d), R, None, ctypes.byref(n))
    if ok:
        assert st == 0 and n.value > 0
    else:
        assert st == -1


def test_workspace_size_matches_system_size(lib):
    """The dense trailing system dominates at 500^3, R = 30: ((N-1)R^2 padded)^2 doubles."""
    from paper_1205_2584_amd import dgn
    n = dgn.workspace_size((500, 500, 500), 30, dgn.torch.float32)
    ntp = ((2 * 900 + 63) // 64) * 64
    assert n > (ntp + 64) * ntp * 8
    assert n < 512 << 20


def test_workspace_size_complex(lib):
    """Complex tensors: the embedded trailing system has twice the real size; R <= 32."""
    from paper_1205_2584_amd import dgn
    torch = dgn.torch
    real = dgn.workspace_size((40, 30, 20), 8, torch.float64)
    cplx = dgn.workspace_size((40, 30, 20), 8, torch.complex128)
    nt = 2 * 2 * 64
    ntp = ((nt + 63) // 64) * 64
    assert cplx > real
    assert cplx > (ntp + 64) * ntp * 8
    assert dgn.workspace_size((40, 30, 20), 32, torch.complex64) > 0
    with pytest.raises(dgn.DgnError):
        dgn.workspace_size((40, 30, 20), 33, torch.complex64)


def test_opts_solver_defaults(lib):
    from paper_1205_2584_amd import dgn
    o = dgn.opts()
    assert o.solver == 0 and o.cg_max_iters == 100 and o.cg_tol == 1e-10 and o.als_sweeps == 0


@pytest.mark.parametrize("dims,R,block,dtype,ok", [
    ((500, 500, 500), 30, 48, "f32", True),
    ((10, 12, 14), 3, 10, "f64", True),
    ((10, 12, 14), 3, 11, "f64", False),     # block > min I_n
    ((100, 100, 100), 30, 81, "f64", False),  # block > 80
    ((10, 12, 14), 11, 11, "f64", False),     # R > min I_n
    ((10, 12, 14), 4, 3, "f64", False),       # block < R
    ((60, 50, 40), 20, 40, "c128", True),
    ((60, 50, 40), 20, 41, "c128", False),    # complex: block <= 40
    ((60, 50, 40), 33, 40, "c64", False),     # complex: R <= 32
])
def test_workspace_size_svd_validates(lib, dims, R, block, dtype, ok):
    from paper_1205_2584_amd import dgn
    torch = dgn.torch
    dt = {"f32": torch.float32, "f64": torch.float64, "c128": torch.complex128, "c64": torch.complex64}[dtype]
    if ok:
        n = dgn.workspace_size_svd(dims, R, block, dt)
        # at least the per-mode Grams (complex: of the doubled embedding)
        f = 2 if dtype.startswith("c") else 1
        assert n >= sum(((f * I + 63) // 64 * 64) ** 2 for I in dims) * 8
    else:
        with pytest.raises(dgn.DgnError) as e:
            dgn.workspace_size_svd(dims, R, block, dt)
        assert e.value.status == -1


def test_opts_mu_rule_default(lib):
    from paper_1205_2584_amd import dgn
    assert dgn.opts().mu_rule == dgn.MU_PAPER == 0 and dgn.MU_NIELSEN == 1


def test_opts_serve_batch_default(lib):
    from paper_1205_2584_amd import dgn
    assert dgn.opts().serve_batch == 1


STRUCTS = {
    "dgn_tensor": ["order", "dims", "dtype", "data"],
    "dgn_opts": ["normalize", "tau", "resid_switch", "y_bf16", "poll_every", "timing", "graph",
                 "als_sweeps", "solver", "cg_max_iters", "cg_tol", "mu_rule", "batched_launch", "serve_batch"],
    "dgn_step_info": ["err2_old", "err2_new", "rho", "denom", "gnorm", "mnorm", "danorm", "cg_iters",
                      "cg_attempt_iters"],
    "dgn_fit_info": ["iters", "accepted", "reason", "resid_iters", "eps", "err2", "mu", "mu0",
                     "cg_trials", "cg_iters", "t_done"],
    "dgn_batch_fit": ["Y", "R", "mu0", "A"],
    "dgn_request": ["Y", "R", "mu0", "tol", "max_iters", "A", "tag"],
    "dgn_result": ["id", "tag", "status", "info", "t_submit", "t_admit", "t_done", "lane", "batch_size"],
    "dgn_batch_tune_entry": ["imax_bucket", "rmax", "launch", "us_per_trial_graph", "us_per_trial_persistent",
                             "sample_fits", "sample_trials"],
}


def test_binding_struct_layout_matches_header(tmp_path):
    """Every struct of the header has the size and field offsets the ctypes binding
    assumes (compiled against include/dgn.h with the host C compiler)."""
    import shutil
    import subprocess
    from paper_1205_2584_amd import dgn
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dgn.h"', "int main(void) {"]
    for s, fields in STRUCTS.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            parts = ln.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for s, fields in STRUCTS.items():
        cls = getattr(dgn, s)
        assert got[(s, "size")] == ctypes.sizeof(cls), s
        assert [n for n, _ in cls._fields_] == fields, s
        for f in fields:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)
