"""The C-ABI library loads on the CPU and exports every entry point that
include/mgrit.h declares, with the documented struct layouts (no compute
calls: there is no GPU here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgrit.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(mgrit_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2104_09404_amd import mgrit

    if not os.path.exists(mgrit.LIB_PATH):
        from paper_2104_09404_amd import build

        build.build()
    return mgrit.load()


def test_header_declares_the_four_named_calls():
    names = declared_functions()
    for n in ("mgrit_phi", "mgrit_relax", "mgrit_residual", "mgrit_cycle"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2104_09404_amd import mgrit

    assert sorted(mgrit.EXPORTED) == declared_functions()


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal the C compiler's
    for include/mgrit.h (a small C program prints them)."""
    import subprocess

    from paper_2104_09404_amd import mgrit

    src = tmp_path / "layout.c"
    checks = {
        "mgrit_scheme": (mgrit.Scheme, ["flux", "k", "stepper", "nx", "a", "eps", "L", "alpha_fixed", "lf_dx_dt",
                                        "numflux"]),
        "mgrit_params": (mgrit.Params, ["nt", "m", "levels", "relax", "cycle", "max_iter", "init", "coarse_guess",
                                        "storage", "sync_every", "dt", "tol", "coarse_integrator"]),
        "mgrit_profile_entry": (mgrit.ProfileEntry, ["launches", "ms", "phi_lines", "cell_steps"]),
        "mgrit_problem": (mgrit.Problem, ["scheme", "nt", "dt", "u0", "u"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "%s"' % HEADER, "int main(void) {"]
    for t, (_, fields) in checks.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (t, t))
        for f in fields:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (t, f, t, f))
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n") if l)
    for t, (cls, fields) in checks.items():
        assert int(out[t]) == C.sizeof(cls), t
        for f in fields:
            assert int(out["%s.%s" % (t, f)]) == getattr(cls, f).offset, (t, f)


def test_validation_errors_without_gpu(lib):
    """Argument checks run on the host before anything touches the device."""
    from paper_2104_09404_amd import mgrit

    bad = mgrit.scheme(4)  # nx < 8
    rc = lib.mgrit_phi(C.byref(bad), 1e-3, None, None, 1, None)
    assert rc == mgrit.MGRIT_EINVAL
    assert b"nx" in lib.mgrit_last_error()
    s = mgrit.scheme(64)
    assert lib.mgrit_phi(C.byref(s), -1.0, None, None, 1, None) == mgrit.MGRIT_EINVAL
    assert lib.mgrit_phi(C.byref(s), 1e-3, None, None, 0, None) == mgrit.MGRIT_OK  # empty input
    assert lib.mgrit_phi(C.byref(s), 1e-3, None, None, 3, None) == mgrit.MGRIT_EINVAL
    big = mgrit.scheme((1 << 20) + 2)
    assert lib.mgrit_phi(C.byref(big), 1e-3, None, None, 1, None) == mgrit.MGRIT_EUNSUPPORTED
    p = mgrit.params(100, 1e-3, 8, 3)  # 100 not divisible by 64
    assert lib.mgrit_workspace_bytes(C.byref(s), C.byref(p)) == 0
    p = mgrit.params(4096, 1e-3, 8, 3)
    n = lib.mgrit_workspace_bytes(C.byref(s), C.byref(p))
    # two coarse levels (513 and 65 nodes, u and g) + side buffer + partials + history
    assert n >= 8 * 64 * (2 * 513 + 2 * 65 + 513)


def test_kernel_config_choice(lib):
    from paper_2104_09404_amd import mgrit

    assert mgrit.kernel_config(64) == (1, 1)
    for nx in (1000, 1024, 4096):
        for nlines in (1, 64, 512):
            cpt, w = mgrit.kernel_config(nx, nlines)
            assert cpt * w * 64 >= nx
    # few lines: more threads per line than for many lines (measured on
    # MI355X; from 1024 cells on, 4 cells x 4 waves wins in both regimes)
    c1, w1 = mgrit.kernel_config(512, 1)
    c2, w2 = mgrit.kernel_config(512, 512)
    assert w1 > w2 and c1 < c2
    assert mgrit.kernel_config(1024, 1) == mgrit.kernel_config(1024, 512) == (4, 4)
    with pytest.raises(mgrit.MgritError):
        mgrit.kernel_config(1 << 20)
    with pytest.raises(mgrit.MgritError):
        mgrit.set_kernel_config(1024, 1024, 4, 2)  # 512 cells do not cover 1024
    mgrit.set_kernel_config(1024, 1024, 8, 4)
    assert mgrit.kernel_config(1024, 512) == (8, 4)
    mgrit.clear_kernel_config()


def test_split_line_choice(lib):
    """Lines up to 4096 cells run on one workgroup; longer ones are split into
    tiles balanced in whole threads: lines of at least 32768 cells that 16
    divides into tiles of up to 8192 cells of 16 per thread, else up to 4096
    cells of 4 per thread when 4 divides the line, else up to 2048 cells of 2
    per thread when it is even, else ragged tiles of up to 2048 cells of 4 per
    thread."""
    from paper_2104_09404_amd import mgrit

    assert mgrit.tiled_config(4096) == (0, 0, 1)
    assert mgrit.tiled_config(65536) == (16, 8, 8)
    assert mgrit.tiled_config(32768) == (16, 8, 4)
    assert mgrit.tiled_config(32772) == (4, 16, 9)
    assert mgrit.tiled_config(16384) == (4, 16, 4)
    assert mgrit.tiled_config(8192) == (4, 16, 2)
    assert mgrit.tiled_config(6002) == (2, 16, 3)
    assert mgrit.tiled_config(6001) == (4, 8, 3)
    assert mgrit.tiled_config(8190) == (2, 16, 4)
    assert mgrit.tiled_config(1 << 20) == (16, 8, 128)
    assert mgrit.tiled_intervals(65536) == 1
    assert mgrit.tiled_config((1 << 20) + 2) == (0, 0, 1)
    mgrit.set_tiled_config(300, 1000, 1, 4)
    assert mgrit.tiled_config(1000) == (1, 4, 4)
    assert mgrit.tiled_config(300) == (1, 4, 2)
    with pytest.raises(mgrit.MgritError):
        mgrit.set_tiled_config(100, 200, 8, 8)  # not compiled as a split-line pair
    mgrit.clear_tiled_config()
    assert mgrit.tiled_config(1000) == (0, 0, 1)
    # the workspace of a split-line problem holds the synchronisation scratch
    s = mgrit.scheme(8192)
    p = mgrit.params(256, 1e-4, 8, 2)
    n_split = lib.mgrit_workspace_bytes(C.byref(s), C.byref(p))
    s2 = mgrit.scheme(4096)
    n_one = lib.mgrit_workspace_bytes(C.byref(s2), C.byref(p))
    assert n_split > 2 * n_one


def test_split_line_latency_choice(lib):
    """One launch over few chunks that forms no residual (serial stepping, the
    coarsest solve, coarse levels) takes 1024-cell tiles of 2 cells per thread
    and 8 waves when the many-chunk shape would occupy fewer than 256
    workgroups, the line is even and at most 131072 cells, and no
    set_tiled_config setting covers it; every other launch keeps the
    many-chunk shape."""
    from paper_2104_09404_amd import mgrit

    mgrit.clear_tiled_config()
    assert mgrit.tiled_launch_config(65536, 1) == (2, 8, 64)
    assert mgrit.tiled_launch_config(65536, 31) == (2, 8, 64)  # 31 x 8 = 248 workgroups
    assert mgrit.tiled_launch_config(65536, 32) == (16, 8, 8)  # 256
    assert mgrit.tiled_launch_config(65536, 1, residual=True) == (16, 8, 8)
    assert mgrit.tiled_launch_config(8192, 127) == (2, 8, 8)
    assert mgrit.tiled_launch_config(8192, 128) == (4, 16, 2)
    assert mgrit.tiled_launch_config(6002, 1) == (2, 8, 6)
    assert mgrit.tiled_launch_config(6001, 1) == (4, 8, 3)  # odd: the ragged default
    assert mgrit.tiled_launch_config(131072, 1) == (2, 8, 128)
    assert mgrit.tiled_launch_config(131074, 1) == (2, 16, 65)  # longer: the default
    assert mgrit.tiled_launch_config(1 << 20, 1) == (16, 8, 128)
    assert mgrit.tiled_launch_config(4096, 1) == (0, 0, 1)  # one workgroup per line
    assert mgrit.tiled_launch_config(65536, 0) == (2, 8, 64)
    with pytest.raises(mgrit.MgritError):
        mgrit.tiled_launch_config(65536, -1)
    mgrit.set_tiled_config(65536, 65536, 4, 16)
    try:
        assert mgrit.tiled_launch_config(65536, 1) == (4, 16, 16)
    finally:
        mgrit.clear_tiled_config()


def test_batch_validation_without_gpu(lib):
    """Batches: the workspace is sized on the host; mixed k or stepper, fewer
    than two levels or an empty batch are rejected before any device call."""
    from paper_2104_09404_amd import mgrit

    p = mgrit.params(0, 0.0, 8, 2, relax=1, max_iter=2, tol=-1.0, storage=1)
    probs = [(mgrit.scheme(256), 1024, 1e-3, None, None), (mgrit.scheme(6002, flux=1, a=0.7), 24008, 1e-4, None, None)]
    n = mgrit.batched_workspace_bytes(probs, p)
    # at least the per-problem coarse level, side buffer, plus the split-line scratch
    assert n > 8 * (2 * 129 * 256 + 2 * 3002 * 6002) + 2 * 1024 * 1024
    arr = mgrit.problem_table(probs)
    assert lib.mgrit_batched_workspace_bytes(arr, 0, C.byref(p)) == 0
    bad = [(mgrit.scheme(256), 1024, 1e-3, None, None), (mgrit.scheme(256, stepper=1), 1024, 1e-3, None, None)]
    assert lib.mgrit_batched_workspace_bytes(mgrit.problem_table(bad), 2, C.byref(p)) == 0
    assert b"same k and stepper" in lib.mgrit_last_error()
    p1 = mgrit.params(0, 0.0, 8, 1)
    assert lib.mgrit_batched_workspace_bytes(arr, 2, C.byref(p1)) == 0
    bad_nt = [(mgrit.scheme(256), 1001, 1e-3, None, None)]
    assert lib.mgrit_batched_workspace_bytes(mgrit.problem_table(bad_nt), 1, C.byref(p)) == 0
    assert b"problem 0" in lib.mgrit_last_error()
    hist = (C.c_double * 8)()
    its = (C.c_int32 * 2)()
    st = (C.c_int32 * 2)()
    rc = lib.mgrit_cycle_batched(arr, 2, C.byref(p), None, 0, hist, its, st, None)
    assert rc == mgrit.MGRIT_EINVAL


def test_autotune_validation_without_gpu(lib):
    """The autotuner checks its arguments on the host: no scratch, or too
    little, is an error before any device call."""
    from paper_2104_09404_amd import mgrit

    s = mgrit.scheme(1024)
    assert lib.mgrit_autotune_scratch_bytes(1024, 512) >= 8 * 1024 * 512
    assert lib.mgrit_autotune_scratch_bytes(4, 1) == 0
    rc = lib.mgrit_autotune(C.byref(s), 512, 8, None, 0, 1, None, None, None, None)
    assert rc == mgrit.MGRIT_EINVAL and b"scratch" in lib.mgrit_last_error()
    assert lib.mgrit_autotune(C.byref(s), 0, 8, None, 0, 1, None, None, None, None) == mgrit.MGRIT_EINVAL


def test_system_validation_without_gpu(lib):
    """Systems: the flux parameter is checked (g > 0, gamma > 1), lines are
    limited to 65536 cells (split above 512: the fewest tiles of at most 510
    cells, with the synchronisation scratch in the cycle workspace), tile
    settings are validated, and the cycle workspace holds D x nx doubles per
    node."""
    from paper_2104_09404_amd import mgrit

    assert lib.mgrit_phi(C.byref(mgrit.shallow_water_scheme(64, g=0.0)), 1e-3, None, None, 1, None) == mgrit.MGRIT_EINVAL
    assert lib.mgrit_phi(C.byref(mgrit.euler_scheme(64, gamma=1.0)), 1e-3, None, None, 1, None) == mgrit.MGRIT_EINVAL
    assert lib.mgrit_phi(C.byref(mgrit.euler_scheme(65537)), 1e-3, None, None, 1, None) == mgrit.MGRIT_EUNSUPPORTED
    assert mgrit.sys_tiles(mgrit.euler_scheme(512)) == 1
    assert mgrit.sys_tiles(mgrit.euler_scheme(513)) == 2
    assert mgrit.sys_tiles(mgrit.shallow_water_scheme(1020, k=3)) == 2
    assert mgrit.sys_tiles(mgrit.shallow_water_scheme(1021)) == 3
    assert mgrit.sys_tiles(mgrit.euler_scheme(65536)) == 129
    with pytest.raises(mgrit.MgritError):
        mgrit.sys_tiles(mgrit.scheme(1000))
    assert lib.mgrit_set_sys_tiles(8, 100, 30) == mgrit.MGRIT_EINVAL  # 0-cell tiles
    assert lib.mgrit_set_sys_tiles(100, 1100, 2) == mgrit.MGRIT_EINVAL  # 550-cell tiles
    assert lib.mgrit_set_sys_tiles(12, 100, 3) == mgrit.MGRIT_OK
    assert mgrit.sys_tiles(mgrit.euler_scheme(64)) == 3
    assert mgrit.sys_tiles(mgrit.euler_scheme(12, k=3)) == 3  # 4-cell tiles hold WENO7's 4 ghost cells
    mgrit.clear_sys_tiles()
    assert mgrit.sys_tiles(mgrit.euler_scheme(64)) == 1
    pb = mgrit.params(512, 1e-3, 8, 2)
    one = lib.mgrit_workspace_bytes(C.byref(mgrit.euler_scheme(512)), C.byref(pb))
    two = lib.mgrit_workspace_bytes(C.byref(mgrit.euler_scheme(513)), C.byref(pb))
    assert two - one > 10e6  # the split-line synchronisation scratch
    assert lib.mgrit_phi(C.byref(mgrit.scheme(64, flux=4)), 1e-3, None, None, 1, None) == mgrit.MGRIT_EINVAL
    p = mgrit.params(512, 1e-3, 8, 2)
    n1 = lib.mgrit_workspace_bytes(C.byref(mgrit.scheme(64)), C.byref(p))
    n3 = lib.mgrit_workspace_bytes(C.byref(mgrit.euler_scheme(64)), C.byref(p))
    assert n3 > 2.5 * n1


def test_noalloc_refuses_oversized_problem_without_gpu(lib):
    """The allocation-free cycle checks its static workspace on the host: a
    problem needing more than MGRIT_NOALLOC_SCRATCH_BYTES (the 65536-cell,
    16384-step V-cycle) is refused before any device call."""
    from paper_2104_09404_amd import mgrit

    s = mgrit.scheme(65536)
    p = mgrit.params(16384, 1e-6, 16, 4, relax=1, max_iter=2, tol=-1.0)
    assert lib.mgrit_workspace_bytes(C.byref(s), C.byref(p)) > mgrit.NOALLOC_SCRATCH_BYTES
    hist = (C.c_double * 3)()
    it = C.c_int32(0)
    assert lib.mgrit_cycle_noalloc(C.byref(s), C.byref(p), None, None, hist, C.byref(it), None) == mgrit.MGRIT_EINVAL
    assert b"static workspace" in lib.mgrit_last_error()
    assert mgrit.NOALLOC_SCRATCH_BYTES == 64 << 20
    text = open(HEADER).read()
    assert "#define MGRIT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in text


def test_split_autotune_validation_without_gpu(lib):
    """The split-line autotuner checks its arguments on the host."""
    from paper_2104_09404_amd import mgrit

    s = mgrit.scheme(8192)
    n = C.c_int32(0)
    args = (None, None, None, None, None)
    assert lib.mgrit_autotune_tiled(C.byref(s), 64, 2, None, 0, 1, *args) == mgrit.MGRIT_EINVAL
    assert b"scratch" in lib.mgrit_last_error()
    assert lib.mgrit_autotune_tiled(C.byref(mgrit.euler_scheme(64)), 64, 2, None, 0, 1, *args) == mgrit.MGRIT_EUNSUPPORTED
    assert lib.mgrit_autotune_tiled(C.byref(s), 0, 2, None, 0, 1, *args) == mgrit.MGRIT_EINVAL
    assert n.value == 0
