"""The C-ABI library builds, loads and exports every symbol the header
declares (CPU only: no compute calls)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "vembddc.h")).read()
    return sorted(set(re.findall(r"\b(vb_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vb_create", "vb_assemble", "vb_setup", "vb_apply", "vb_pcg_solve",
                     "vb_get_local_solution", "vb_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2304_09770_amd.build import build
        build()
    lib = binding.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(binding.exported_symbols()) == _declared()


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    from paper_2304_09770_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.load()


def test_binding_structs_match_the_header(tmp_path):
    """Every struct of the header has the same size and field offsets in the
    ctypes binding as in C (a gcc probe of include/vembddc.h)."""
    import ctypes
    import shutil
    import subprocess

    from paper_2304_09770_amd import binding
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    structs = [getattr(binding, n) for n in ("vb_options", "vb_problem", "vb_face_info",
                                             "vb_kernel_stat", "vb_subdomain", "vb_entity",
                                             "vb_solve_info")]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vembddc.h"', "int main(void) {"]
    for S in structs:
        n = S.__name__
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (n, n))
        for f, _ in S._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (n, f, n, f))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for S in structs:
        n = S.__name__
        assert got[(n, "sizeof")] == ctypes.sizeof(S), n
        for f, _ in S._fields_:
            assert got[(n, f)] == getattr(S, f).offset, (n, f)
    # and no field of the header is missing from the binding
    txt = open(os.path.join(ROOT, "include", "vembddc.h")).read()
    for S in structs:
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (S.__name__, S.__name__), txt, re.S)
        assert body, S.__name__
        decl = re.sub(r"/\*.*?\*/", "", body.group(1), flags=re.S)
        names = re.findall(r"(\w+)\s*(?:,|;)", decl)
        assert sorted(names) == sorted(f for f, _ in S._fields_), S.__name__


@pytest.mark.parametrize("kw", [dict(panel=48), dict(precision=7), dict(scaling=3),
                                dict(setup_mem_limit=-1.0), dict(local_mem_limit=float("nan")),
                                dict(tol=float("nan")), dict(tol=float("inf")),
                                dict(svd_tol=float("nan")), dict(adaptive_theta=-1.0),
                                dict(adaptive_theta=float("nan")), dict(fp32_pivot_min=-1.0),
                                dict(fp32_pivot_min=float("nan")),
                                dict(fp32_pivot_min=float("inf")), dict(tune_factor=3),
                                dict(tune_factor=-1), dict(inner_tol=1.0), dict(inner_tol=-1e-3),
                                dict(inner_tol=float("nan"))])
def test_bad_options_are_rejected_on_the_host(kw):
    """vb_create checks its options before any HIP call, so this runs without
    a GPU."""
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2304_09770_amd.build import build
        build()
    with pytest.raises(binding.VBError) as e:
        binding.vb_create(**kw)
    assert e.value.code == -1


def test_binding_refuses_host_mistyped_or_short_tensors():
    """Device arguments are checked before the library is called: a host
    tensor, a wrong element type or a short vector raises instead of
    handing the kernels a bad address.  A stand-in object plays the GPU
    tensor, so no device is needed."""
    torch = pytest.importorskip("torch")
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2304_09770_amd.build import build
        build()

    class OnGpu:
        is_cuda = True

        def __init__(self, dtype, n, contiguous=True):
            self.dtype, self.n, self.c = dtype, n, contiguous

        def is_contiguous(self):
            return self.c

        def numel(self):
            return self.n

        def data_ptr(self):
            return 4096

    with pytest.raises(ValueError):
        binding.vb_rhs(None, torch.zeros(4, dtype=torch.float64))  # host memory
    with pytest.raises(TypeError):
        binding._ptr(OnGpu(torch.float32, 10), "float64")
    with pytest.raises(ValueError):
        binding._ptr(OnGpu(torch.float64, 3), "float64", 10)
    with pytest.raises(ValueError):
        binding._ptr(OnGpu(torch.float64, 10, contiguous=False), "float64")
    assert binding._ptr(OnGpu(torch.float64, 10), "float64", 10) == 4096
    assert binding._ptr(12288) == 12288 and binding._ptr(None) is None
