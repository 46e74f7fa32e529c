"""The C-ABI library loads, exports every entry point include/emc.h declares,
and rejects invalid arguments on the host before launching anything (these
calls never reach the GPU, so they run without one)."""
import ctypes
import os
import re

import pytest

from paper_1409_4256_amd import emc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return emc.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "emc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(emc_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(emc.EXPORTS)


def test_strides(lib):
    assert emc.emc_pix_stride(16384) == 16384
    assert emc.emc_pix_stride(1024) == 1024
    assert emc.emc_pix_stride(529) == 768
    assert emc.emc_data_stride(100000) == 100096
    assert emc.emc_data_stride(0) == 0


def _pb(**kw):
    fake = 1 << 20  # never dereferenced: validation fails before any launch
    d = dict(grid_n=32, n_pix=1024, n_rot=1000, n_data=1000, precision=0, reserved=0,
             q=fake, mask=fake, quat=fake, log_w=fake, scatter=None)
    d.update(kw)
    return emc.Problem(*[d[k] for k, _ in emc.Problem._fields_])


@pytest.mark.parametrize("prec,elem", [(0, 4), (1, 2)])
def test_buffer_sizes_config2(lib, prec, elem):
    pb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000, precision=prec)
    n = ctypes.c_size_t()
    assert lib.emc_workspace_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    slices = 25000 * 16384 * 4
    g = 25000 * 100096 * 4
    p = 0 if prec == 0 else 25000 * 100096 * 2          # FP32 responsibilities overwrite G
    copies = 16 * 128 ** 3 * 8                           # per-XCD numerator and denominator grids
    assert slices + g + p + copies < n.value < slices + g + p + copies + 64 * 2 ** 20
    assert lib.emc_compress_workspace_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    assert n.value == copies
    assert lib.emc_frames_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    assert n.value == (100000 * 16384 + 16384 * 100096) * elem
    assert lib.emc_slices_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    assert n.value == slices


@pytest.mark.parametrize("field,value,status", [
    ("grid_n", 1, emc.EMC_ERR_INVALID_ARG), ("grid_n", 2000, emc.EMC_ERR_INVALID_ARG),
    ("n_pix", 0, emc.EMC_ERR_INVALID_ARG), ("n_rot", 0, emc.EMC_ERR_INVALID_ARG),
    ("n_data", -1, emc.EMC_ERR_INVALID_ARG), ("reserved", 3, emc.EMC_ERR_INVALID_ARG),
    ("precision", 7, emc.EMC_ERR_INVALID_ARG), ("precision", -1, emc.EMC_ERR_INVALID_ARG),
])
def test_problem_validation(lib, field, value, status):
    pb = _pb(**{field: value})
    n = ctypes.c_size_t()
    assert lib.emc_workspace_bytes(ctypes.byref(pb), ctypes.byref(n)) == status
    assert len(lib.emc_last_error()) > 0


def test_null_and_misaligned_pointers_rejected(lib):
    pb = _pb()
    z = ctypes.c_void_p(0)
    a = ctypes.c_void_p(1 << 20)
    assert lib.emc_expand(ctypes.byref(pb), z, a, a, a, z, z) == emc.EMC_ERR_INVALID_ARG
    assert b"model" in lib.emc_last_error()
    assert lib.emc_expand(ctypes.byref(pb), a, ctypes.c_void_p((1 << 20) + 4), a, a, z, z) == emc.EMC_ERR_INVALID_ARG
    assert b"aligned" in lib.emc_last_error()
    assert lib.emc_expand(ctypes.byref(_pb(quat=0)), a, a, a, a, z, z) == emc.EMC_ERR_INVALID_ARG
    # BF16 form needs the per-rotation scale output
    assert lib.emc_expand(ctypes.byref(_pb(precision=1)), a, a, a, a, z, z) == emc.EMC_ERR_INVALID_ARG
    assert b"scale" in lib.emc_last_error()
    # BF16 responsibilities may not overwrite G
    pb16 = _pb(precision=1)
    assert lib.emc_responsibilities(ctypes.byref(pb16), a, a, a, 0, a, a, a, a, z) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_responsibilities(ctypes.byref(pb), a, a, a, 9, a, a, a, a, z) == emc.EMC_ERR_INVALID_ARG


def test_workspace_checks(lib):
    pb = _pb()
    a = ctypes.c_void_p(1 << 20)
    need = ctypes.c_size_t()
    lib.emc_workspace_bytes(ctypes.byref(pb), ctypes.byref(need))
    st = lib.emc_iterate(ctypes.byref(pb), a, a, a, a, None, a, ctypes.c_size_t(need.value - 1), None)
    assert st == emc.EMC_ERR_WORKSPACE
    assert b"needs" in lib.emc_last_error()
    st = lib.emc_iterate(ctypes.byref(pb), a, a, a, a, None, None, need, None)
    assert st == emc.EMC_ERR_WORKSPACE
    st = lib.emc_iterate(ctypes.byref(pb), a, a, a, a, None, ctypes.c_void_p((1 << 20) + 16), need, None)
    assert st == emc.EMC_ERR_WORKSPACE


def test_noalloc_refuses_problems_beyond_its_static_buffer(lib):
    """emc_iterate_noalloc checks the problem's workspace against its fixed buffer
    before looking the buffer up or launching anything."""
    a = ctypes.c_void_p(1 << 20)
    big = _pb(grid_n=64, n_pix=4096, n_rot=4000, n_data=4000)
    need = ctypes.c_size_t()
    assert lib.emc_workspace_bytes(ctypes.byref(big), ctypes.byref(need)) == emc.EMC_OK
    assert need.value > emc.EMC_SCRATCH_MAX_BYTES
    assert lib.emc_iterate_noalloc(ctypes.byref(big), a, a, a, a, None, None) == emc.EMC_ERR_WORKSPACE
    assert b"static scratch" in lib.emc_last_error()
    assert lib.emc_iterate_noalloc(ctypes.byref(_pb()), None, a, a, a, None, None) == emc.EMC_ERR_INVALID_ARG


def test_validate_argument_checks(lib):
    a = ctypes.c_void_p(1 << 20)
    assert lib.emc_validate(ctypes.byref(_pb()), a, None, None) == emc.EMC_ERR_INVALID_ARG
    assert b"flags" in lib.emc_last_error()
    assert lib.emc_validate(ctypes.byref(_pb(quat=0)), a, a, None) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_validate(ctypes.byref(_pb()), ctypes.c_void_p((1 << 20) + 2), a, None) == emc.EMC_ERR_INVALID_ARG


def test_compress_workspace_checks(lib):
    pb = _pb()
    a = ctypes.c_void_p(1 << 20)
    need = ctypes.c_size_t()
    lib.emc_compress_workspace_bytes(ctypes.byref(pb), ctypes.byref(need))
    st = lib.emc_compress(ctypes.byref(pb), a, a, a, a, a, a, 0, a, ctypes.c_size_t(need.value - 1), None)
    assert st == emc.EMC_ERR_WORKSPACE
    st = lib.emc_compress(ctypes.byref(pb), a, a, a, a, a, a, 0, ctypes.c_void_p((1 << 20) + 8), need, None)
    assert st == emc.EMC_ERR_WORKSPACE


def test_python_binding_raises_emc_error(lib):
    with pytest.raises(emc.EmcError) as e:
        emc._check(emc.EMC_ERR_INVALID_ARG)
    assert e.value.status == emc.EMC_ERR_INVALID_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of emc_problem, emc_proposal and emc_scatter_plan, from the C
    compiler reading include/emc.h, equal the Python binding's mirrors."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs gcc and the ROCm headers")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "emc.h"', "int main(void) {"]
    structs = (("emc_problem", emc.Problem), ("emc_proposal", emc.Proposal), ("emc_scatter_plan", emc.ScatterPlan),
               ("emc_proposed_view", emc.ProposedView))
    for cname, cls in structs:
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, cls in structs:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f


def test_proposal_argument_checks(lib):
    pb = _pb(precision=1)
    n = ctypes.c_size_t()
    assert lib.emc_proposal_bytes(ctypes.byref(pb), 2000, 256, 20, 1 << 20, ctypes.byref(n)) == emc.EMC_OK
    assert n.value > 0
    assert lib.emc_proposal_bytes(ctypes.byref(pb), 2000, 257, 20, 1 << 20, ctypes.byref(n)) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_proposal_bytes(ctypes.byref(pb), 0, 8, 20, 1 << 20, ctypes.byref(n)) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_proposal_bytes(ctypes.byref(pb), 2000, 8, 2000, 1 << 20, ctypes.byref(n)) == emc.EMC_ERR_INVALID_ARG
    a = ctypes.c_void_p(1 << 20)
    assert lib.emc_topk_union(a, 300, a, 300, 10, 2000, a, None) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_topk_union(a, 0, a, 0, 10, 2000, a, None) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_topk_union(a, 8, a, 8, 0, 2000, a, None) == emc.EMC_OK       # no rows: nothing launched
    assert lib.emc_cell_topk(a, 10, 100, 101, a, None) == emc.EMC_ERR_INVALID_ARG
    assert lib.emc_cell_topk(a, 0, 100, 10, a, None) == emc.EMC_OK
    # an inconsistent plan is refused before anything runs
    plan = emc.Proposal()
    assert lib.emc_proposed_workspace_bytes(ctypes.byref(pb), ctypes.byref(plan), ctypes.byref(n)) == \
        emc.EMC_ERR_INVALID_ARG


def _consistent_plan(pb, n_audit=20, **kw):
    fake = 1 << 20  # never dereferenced
    n_cand = pb.n_data - n_audit
    d = dict(n_cells=2000, k_top=128, n_cand=n_cand, n_audit=n_audit, words=63, n_bands=pb.n_pix // 128 if
             pb.n_pix % 256 == 0 else (pb.n_pix + 255) // 256 * 2, n_groups=2000, n_tiles=8 * 100, n_g=1 << 20,
             n_chunks=1 << 16, n_dense=4, n_packs=1, ld_dense=(n_cand + 255) // 256 * 256,
             n_rot=pb.n_rot, n_pix=pb.n_pix, quat=pb.quat, mask=pb.mask)
    d.update(kw)
    plan = emc.Proposal()
    for f, _ in emc.Proposal._fields_:
        setattr(plan, f, d.get(f, fake))
    return plan


def test_proposal_plan_must_match_the_problem(lib):
    """A plan whose sizes are consistent but which was built for another rotation set
    or detector is refused before any launch (its rotation lists would index outside
    this problem's slices)."""
    pb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000, precision=1)
    n = ctypes.c_size_t()
    good = _consistent_plan(pb)
    assert lib.emc_proposed_workspace_bytes(ctypes.byref(pb), ctypes.byref(good), ctypes.byref(n)) == emc.EMC_OK
    v = emc.ProposedView()
    assert lib.emc_proposed_workspace_view(ctypes.byref(pb), ctypes.byref(good), ctypes.byref(v)) == emc.EMC_OK
    assert 0 <= v.S < v.G < v.P < v.Ga < v.Pa < n.value
    a = ctypes.c_void_p(1 << 20)
    for field, value in (("n_rot", 30000), ("n_rot", 20000), ("n_pix", 8192), ("quat", (1 << 20) + 4096),
                         ("mask", (1 << 20) + 4096)):
        bad = _consistent_plan(pb, **{field: value})
        assert lib.emc_proposed_workspace_bytes(ctypes.byref(pb), ctypes.byref(bad), ctypes.byref(n)) == \
            emc.EMC_ERR_INVALID_ARG, field
        assert "another rotation set" in lib.emc_last_error().decode()
        assert lib.emc_iterate_proposed(ctypes.byref(pb), ctypes.byref(bad), a, a, a, a, a, a, ctypes.c_size_t(1 << 40),
                                        None, None) == emc.EMC_ERR_INVALID_ARG, field
        assert lib.emc_proposed_accumulate(ctypes.byref(pb), ctypes.byref(bad), a, a, a, a, 0, 0.98, a, a, a,
                                           ctypes.c_size_t(1 << 40), None, None) == emc.EMC_ERR_INVALID_ARG, field
    # a NaN acceptance threshold is refused
    assert lib.emc_proposed_accumulate(ctypes.byref(pb), ctypes.byref(good), a, a, a, a, 0, float("nan"), a, a, a,
                                       ctypes.c_size_t(1 << 40), None, None) == emc.EMC_ERR_INVALID_ARG


def test_proposal_plan_bytes_config2(lib):
    """Plan buffer of the 128^3 workload with 128-entry lists stays modest."""
    pb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000, precision=1)
    n = ctypes.c_size_t()
    assert lib.emc_proposal_bytes(ctypes.byref(pb), 2000, 128, 2000, 200_000_000, ctypes.byref(n)) == emc.EMC_OK
    assert n.value < 3 * 2 ** 30


def _fake_plan(pb, **kw):
    d = dict(grid_n=pb.grid_n, n_pix=pb.n_pix, n_rot=pb.n_rot, brick=16, n_bricks=((pb.grid_n + 15) // 16) ** 3,
             n_groups=(pb.n_pix + 63) // 64, chunk=2048, reserved=0, n_visits=10, n_items=1, bytes=0,
             visits=1 << 20, items=1 << 20, rot=1 << 20, q=pb.q, mask=pb.mask, quat=pb.quat)
    d.update(kw)
    return emc.ScatterPlan(*[d[k] for k, _ in emc.ScatterPlan._fields_])


def test_scatter_plan_argument_checks(lib):
    """Brick-major c-step plan: sizes, and plans that do not fit the geometry are refused."""
    pb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000)
    n = ctypes.c_size_t()
    assert lib.emc_scatter_plan_min_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    # 512 brick counters, 513 offsets, the FP64 R_j table, each rounded up to 256 bytes
    assert n.value == 2048 + 4352 + -(-25000 * 72 // 256) * 256
    a = ctypes.c_void_p(1 << 20)
    plan = emc.ScatterPlan()
    assert lib.emc_scatter_plan_build(ctypes.byref(pb), 5, a, n, ctypes.byref(plan), None) == emc.EMC_ERR_INVALID_ARG
    assert b"chunk" in lib.emc_last_error()
    big = _pb(n_rot=2 ** 31 - 1)
    assert lib.emc_scatter_plan_build(ctypes.byref(big), 0, a, n, ctypes.byref(plan), None) == emc.EMC_ERR_UNSUPPORTED
    assert lib.emc_scatter_plan_build(ctypes.byref(pb), 0, ctypes.c_void_p((1 << 20) + 8), n, ctypes.byref(plan),
                                      None) == emc.EMC_ERR_INVALID_ARG
    # with a plan the c-step needs no grid copies
    good = _fake_plan(pb)
    pbs = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000, scatter=ctypes.addressof(good))
    assert lib.emc_compress_workspace_bytes(ctypes.byref(pbs), ctypes.byref(n)) == emc.EMC_OK
    assert n.value == 0
    w0, w1 = ctypes.c_size_t(), ctypes.c_size_t()
    lib.emc_workspace_bytes(ctypes.byref(pb), ctypes.byref(w0))
    lib.emc_workspace_bytes(ctypes.byref(pbs), ctypes.byref(w1))
    assert w0.value - w1.value == 16 * 128 ** 3 * 8
    # a plan of another geometry, or an inconsistent one, is refused before any launch
    for bad in (_fake_plan(pb, grid_n=64), _fake_plan(pb, n_rot=24999), _fake_plan(pb, quat=1 << 21),
                _fake_plan(pb, brick=8), _fake_plan(pb, n_groups=3), _fake_plan(pb, items=0)):
        pbb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000, scatter=ctypes.addressof(bad))
        st = lib.emc_compress(ctypes.byref(pbb), a, a, a, a, a, a, 0, None, 0, None)
        assert st == emc.EMC_ERR_INVALID_ARG
        assert b"scatter plan" in lib.emc_last_error()


def test_gaussian_argument_checks(lib):
    """Gaussian-model iteration: sizes, sigma, form and workspace are checked before any launch."""
    pb = _pb(grid_n=128, n_pix=16384, n_rot=25000, n_data=100000)
    n = ctypes.c_size_t()
    assert lib.emc_gaussian_workspace_bytes(ctypes.byref(pb), ctypes.byref(n)) == emc.EMC_OK
    slices, g = 25000 * 16384 * 4, 25000 * 100096 * 4
    assert slices + 2 * g < n.value < slices + 2 * g + 16 * 128 ** 3 * 8 + 64 * 2 ** 20
    a = ctypes.c_void_p(1 << 20)
    small = _pb()
    lib.emc_gaussian_workspace_bytes(ctypes.byref(small), ctypes.byref(n))
    for sigma in (0.0, -1.0, float("inf"), float("nan")):
        st = lib.emc_iterate_gaussian(ctypes.byref(small), sigma, a, a, a, 1, a, a, None, a, n, None)
        assert st == emc.EMC_ERR_INVALID_ARG
        assert b"sigma" in lib.emc_last_error()
    st = lib.emc_iterate_gaussian(ctypes.byref(_pb(precision=1)), 1.0, a, a, a, 1, a, a, None, a, n, None)
    assert st == emc.EMC_ERR_UNSUPPORTED
    st = lib.emc_iterate_gaussian(ctypes.byref(small), 1.0, a, a, a, 1, a, a, None, a,
                                  ctypes.c_size_t(n.value - 1), None)
    assert st == emc.EMC_ERR_WORKSPACE
    st = lib.emc_iterate_gaussian(ctypes.byref(small), 1.0, a, a, None, 1, a, a, None, a, n, None)
    assert st == emc.EMC_ERR_INVALID_ARG and b"phi" in lib.emc_last_error()
