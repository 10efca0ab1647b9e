"""The C-ABI library builds, loads and exports every symbol of include/cavity.h.

Runs without a GPU: only host-side entry points that touch no device are
called (workspace sizing and argument validation).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cavity.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cavity_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    lib = os.path.join(ROOT, "paper_0809_3098_amd", "libcavity.so")
    if not os.path.exists(lib):
        from paper_0809_3098_amd.build import build
        build()
    import paper_0809_3098_amd.cavity as b
    return b


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ("cavity_create", "cavity_step", "cavity_poisson", "cavity_fields",
              "cavity_destroy", "cavity_last_error", "cavity_workspace_bytes"):
        assert f in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(binding.EXPORTED) <= set(_declared_functions())


def test_struct_layout_matches_header(binding):
    # offsets of the C structs as laid out by a C compiler for this header
    assert ctypes.sizeof(binding.cavity_params) == 96
    assert binding.cavity_params.omega0.offset == 72
    assert binding.cavity_params.fixed_sweeps.offset == 88
    assert ctypes.sizeof(binding.cavity_stats) == 88
    assert ctypes.sizeof(binding.cavity_poisson_info) == 24


def test_struct_layout_matches_c_compiler(binding, tmp_path):
    """ctypes layouts against offsetof/sizeof from gcc on the header itself."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    checks = []
    for sname in ("cavity_params", "cavity_stats", "cavity_poisson_info", "cavity_tuning"):
        cls = getattr(binding, sname)
        checks.append((f"sizeof({sname})", ctypes.sizeof(cls)))
        for fname, _ in cls._fields_:
            checks.append((f"offsetof({sname}, {fname})", getattr(cls, fname).offset))
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", (size_t){e});\n' for e, _ in checks)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cavity.h"\n'
                   f"int main(void) {{\n{body}  return 0;\n}}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    for (expr, want), g in zip(checks, got):
        assert g == want, expr


def test_workspace_bytes_scales_with_grid(binding):
    P = binding.Params
    small = binding.cavity_workspace_bytes([P(n=64).to_c()])
    big = binding.cavity_workspace_bytes([P(n=1024).to_c()])
    assert big > 20 * small
    # eight FP64 fields of 1024 x 1024 at least
    assert big >= 8 * 1024 * 1024 * 8
    # (without the warm-start history, whose default depth depends on precision)
    fp64 = binding.cavity_workspace_bytes([P(n=1024, warm_start=1).to_c()])
    mixed = binding.cavity_workspace_bytes([P(n=1024, precision=binding.CAVITY_MIXED,
                                              warm_start=1).to_c()])
    assert mixed >= fp64 + 3 * 1024 * 1024 * 4
    two = binding.cavity_workspace_bytes([P(n=64).to_c(), P(n=1024).to_c()])
    # one shared handle area (descriptors, barrier flags) instead of two
    assert small + big - 600 * 1024 <= two < small + big


def test_workspace_bytes_holds_the_warm_start_history(binding):
    """Extrapolated warm starts keep 5 fields (one per SSPRK stage) per level,
    plus a step counter and the weight table (256 + 768 bytes)."""
    P = binding.Params
    field = 1024 * 1024 * 8   # 1024 nodes a side, pitch 1024
    extra = 256 + 768
    prev = binding.cavity_workspace_bytes([P(n=1024, warm_start=1).to_c()])
    for levels in range(2, binding.CAVITY_WARM_LEVELS_MAX + 1):
        got = binding.cavity_workspace_bytes([P(n=1024, warm_start=levels).to_c()])
        assert got - prev == 5 * levels * field + extra
    default = binding.cavity_workspace_bytes([P(n=1024).to_c()])
    assert default - prev == 5 * binding.CAVITY_WARM_LEVELS_FP64 * field + extra
    mixed_prev = binding.cavity_workspace_bytes(
        [P(n=1024, precision=binding.CAVITY_MIXED, warm_start=1).to_c()])
    mixed = binding.cavity_workspace_bytes([P(n=1024, precision=binding.CAVITY_MIXED).to_c()])
    assert mixed - mixed_prev == 5 * binding.CAVITY_WARM_LEVELS_MIXED * field + extra
    # the coupled mode starts every stage from the previous stage's psi
    fixed = binding.cavity_workspace_bytes([P(n=1024, fixed_sweeps=8).to_c()])
    assert fixed == prev


@pytest.mark.parametrize("kw,msg", [
    (dict(n=4), "n ="),
    (dict(n=64, re=0.0), "re must"),
    (dict(n=64, re=float("nan")), "non-finite"),
    (dict(n=64, u_lid=0.0), "dt must"),
    (dict(n=64, sor_omega=2.0), "sor_omega"),
    (dict(n=64, precision=7), "precision"),
    (dict(n=64, resume=1), "resume"),
    (dict(n=64, fixed_sweeps=-1), "fixed_sweeps"),
    (dict(n=64, fixed_sweeps=4, precision=1), "fixed_sweeps needs"),
    (dict(n=64, warm_start=9), "warm_start"),
    (dict(n=64, warm_start=-1), "warm_start"),
    (dict(n=64, fixed_sweeps=4, warm_start=2), "warm_start extrapolation"),
])
def test_invalid_parameters_are_rejected(binding, kw, msg):
    with pytest.raises(binding.CavityError) as e:
        binding.cavity_workspace_bytes([binding.Params(**kw).to_c()])
    assert e.value.code == binding.CAVITY_EINVAL
    assert msg in e.value.message


def test_create_rejects_before_touching_a_device(binding):
    P = binding.Params
    with pytest.raises(binding.CavityError) as e:
        binding.cavity_create([P(n=3).to_c()], 256, 1 << 20, 0)
    assert e.value.code == binding.CAVITY_EINVAL
    with pytest.raises(binding.CavityError) as e:
        binding.cavity_create([P(n=64).to_c()], 256 + 8, 1 << 30, 0)
    assert "aligned" in e.value.message
    with pytest.raises(binding.CavityError) as e:
        binding.cavity_create([P(n=64).to_c()], 256, 16, 0)
    assert e.value.code == binding.CAVITY_ENOMEM
    with pytest.raises(binding.CavityError) as e:
        binding.cavity_step(0, 1)
    assert e.value.code == binding.CAVITY_EINVAL


def test_noalloc_solve_rejects_before_touching_a_device(binding):
    """The allocation-free solve checks its arguments before any HIP call."""
    for n, ptr in ((1025, 256), (4, 256), (64, 0)):
        with pytest.raises(binding.CavityError) as e:
            binding.cavity_poisson_noalloc(n, ptr, ptr, 0)
        assert e.value.code == binding.CAVITY_EINVAL
