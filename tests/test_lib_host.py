"""Host-side checks of libkl that need no GPU: the library loads and exports
every entry point declared in include/kl.h, the layout rules, argument
checks, and the wisdom-record selection heuristic."""
import json
import os
import re

import pytest

from paper_2303_12374_amd import kl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "kl.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(kl_[a-z0-9_]+)\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 25
    for n in names:
        assert hasattr(kl._lib, n), f"{n} declared in kl.h but not exported by libkl.so"
    assert set(names) == set(kl.DECLARED), "binding and header disagree"


def test_version_and_no_error():
    assert "gfx950" in kl.kl_version()


@pytest.mark.parametrize("dtype,s", [(kl.F32, 4), (kl.F64, 8)])
@pytest.mark.parametrize("shape", [(512, 512, 512), (1024, 1024, 128), (37, 23, 19), (1, 1, 2), (96, 64, 32)])
def test_layout_alignment(dtype, s, shape):
    itot, jtot, ktot = shape
    off, js, ks, alloc = kl.kl_layout(itot, jtot, ktot, dtype)
    assert ((off + 1) * s) % 128 == 0, "first interior element of row 0 on a 128-byte line"
    assert (js * s) % 128 == 0 and js >= itot + 2
    assert ks == js * (jtot + 2)
    assert alloc >= off + ks * (ktot + 2)
    # x ghosts of rows j and j+1 share one 128-byte line
    last_ghost = off + itot + 1
    next_first = off + js
    assert (last_ghost * s) // 128 == (next_first * s) // 128


@pytest.mark.parametrize("dtype,s", [(kl.F32, 4), (kl.F64, 8)])
@pytest.mark.parametrize("shape", [(512, 512, 512), (37, 23, 19), (1, 1, 2), (2, 3, 4)])
def test_layout_three_ghost_cells(dtype, s, shape):
    """gc = 3: interior rows start on a 128-byte line, the first ghost cell
    (1-3, 1-3, 0) has a non-negative index, the last one fits the allocation,
    and rows / planes hold itot+6 / jtot+6 cells."""
    itot, jtot, ktot = shape
    off, js, ks, alloc = kl.kl_layout_gc(itot, jtot, ktot, dtype, 3)
    assert ((off + 1) * s) % 128 == 0
    assert (js * s) % 128 == 0 and js >= itot + 6
    assert ks == js * (jtot + 6)
    assert off + (1 - 3) + (1 - 3) * js >= 0
    assert off + (itot + 3) + (jtot + 3) * js + (ktot + 1) * ks < alloc
    assert kl.kl_layout_gc(itot, jtot, ktot, dtype, 1) == kl.kl_layout(itot, jtot, ktot, dtype)


def test_layout_rejects_bad_sizes():
    with pytest.raises(kl.KLError) as e:
        kl.kl_layout(0, 4, 4, kl.F32)
    assert e.value.code == kl.ERR_INVALID
    with pytest.raises(kl.KLError):
        kl.kl_layout(4, 4, 4, 7)


def test_argument_checks_need_no_device():
    g = kl.kl_grid_t(8, 8, 8, 1, 0, 10, 100, 8.0, 8.0, 16, 16, kl.F32, 0)
    for bad in (dict(gc=2), dict(itot=0), dict(jstride=5), dict(kstride=50), dict(dtype=3), dict(bc=9),
                dict(dzi=None), dict(ktot=1)):
        gg = kl.kl_grid_t.from_buffer_copy(g)
        for k, v in bad.items():
            setattr(gg, k, v)
        with pytest.raises(kl.KLError) as e:
            kl.kl_advec_u(gg, 1, 1, 1, 1, stream=0)
        assert e.value.code == kl.ERR_INVALID
    with pytest.raises(kl.KLError):
        kl.kl_advec_u(g, None, 1, 1, 1, stream=0)
    with pytest.raises(kl.KLError):
        kl.kl_reduce_fp64(g, 5, 1, 1, 1, 1, stream=0)


def test_new_scheme_argument_checks_need_no_device():
    """advec_u_2i5 refuses a grid with one ghost cell; diff_smag refuses a
    NULL eddy viscosity; gc must be 1 or 3 (all before any device work)."""
    off, js, ks, _ = kl.kl_layout(8, 8, 8, kl.F32)
    g1 = kl.kl_grid_t(8, 8, 8, 1, off, js, ks, 8.0, 8.0, 16, 16, kl.F32, 0)
    with pytest.raises(kl.KLError) as e:
        kl.kl_advec_u_2i5(g1, 64, 64, 64, 64, stream=0)
    assert e.value.code == kl.ERR_INVALID and "gc" in str(e.value)
    with pytest.raises(kl.KLError) as e:
        kl.kl_diff_smag(g1, 64, 64, 64, 64, 64, 64, None, stream=0)
    assert e.value.code == kl.ERR_INVALID
    off3, js3, ks3, _ = kl.kl_layout_gc(8, 8, 8, kl.F32, 3)
    g3 = kl.kl_grid_t(8, 8, 8, 3, off3, js3, ks3, 8.0, 8.0, 16, 16, kl.F32, 0)
    bad = kl.kl_grid_t.from_buffer_copy(g3)
    bad.off = 10  # first ghost cells would lie before the buffer
    with pytest.raises(kl.KLError):
        kl.kl_fill_ghosts(bad, 64, 64, 64, stream=0)
    with pytest.raises(kl.KLError):
        kl.kl_layout_gc(8, 8, 8, kl.F32, 2)


def test_variant_registry():
    for dt in (kl.F32, kl.F64):
        for kern in (kl.ADVEC_U, kl.DIFF_UVW):
            n = kl.kl_num_variants(kern, dt)
            assert n > 10
            assert kl.kl_variant_name(kern, dt, 0) == "default"
            names = [kl.kl_variant_name(kern, dt, i) for i in range(n)]
            assert len(set(names)) == n
    with pytest.raises(kl.KLError):
        kl.kl_variant_name(kl.ADVEC_U, kl.F32, 10 ** 6)


def _rec(variant, size, device="AMD Instinct MI355X", arch="gfx950", dtype="f32", kernel="advec_u", cu=None):
    r = {"kernel": kernel, "dtype": dtype, "problem_size": list(size), "device": device,
         "arch": arch, "variant": variant, "time_ms": 1.0}
    if cu is not None:
        r["cu_count"] = cu
    return json.dumps(r)


def test_wisdom_selection_levels(tmp_path):
    """The five cases of the selection heuristic (Section "Kernel Selection
    and Compilation"), on synthetic records."""
    v = [kl.kl_variant_name(kl.ADVEC_U, kl.F32, i) for i in range(1, 6)]
    d = str(tmp_path)
    look = lambda dev, arch, size, dtype=kl.F32: kl.kl_wisdom_lookup(d, kl.ADVEC_U, dtype, dev, arch, *size)
    # 5: missing file -> default
    assert look("AMD Instinct MI355X", "gfx950", (256, 256, 256)) == ("default", 5)
    lines = [
        _rec(v[0], (256, 256, 256)),
        _rec(v[1], (512, 512, 512)),
        _rec(v[2], (128, 128, 128), device="AMD Instinct MI350X"),
        _rec(v[3], (64, 64, 64), device="Other GPU", arch="gfx942"),
        "this line is not json",
        _rec(v[4], (256, 256, 256), dtype="f64"),
        _rec("no_such_configuration", (100, 100, 100)),
    ]
    (tmp_path / "advec_u.wisdom").write_text("\n".join(lines) + "\n")
    # 1: exact GPU and size
    assert look("AMD Instinct MI355X", "gfx950", (256, 256, 256)) == (v[0], 1)
    # 2: same GPU, nearest size (Euclidean): (400,400,400) is nearer 512^3
    assert look("AMD Instinct MI355X", "gfx950", (400, 400, 400)) == (v[1], 2)
    assert look("AMD Instinct MI355X", "gfx950", (300, 300, 300)) == (v[0], 2)
    # 3: other GPU of the same architecture: nearest among gfx950 records
    assert look("AMD Instinct MI999", "gfx950", (120, 120, 120)) == (v[2], 3)
    # 4: unknown architecture: nearest of all records
    assert look("Some GPU", "gfx1100", (60, 60, 60)) == (v[3], 4)
    # dtype must match: the only f64 record is chosen for f64 whatever its size
    assert look("AMD Instinct MI355X", "gfx950", (32, 32, 32), dtype=kl.F64) == (v[4], 2)
    # a later record for the same GPU and size supersedes the earlier one
    with open(tmp_path / "advec_u.wisdom", "a") as f:
        f.write(_rec(v[2], (256, 256, 256)) + "\n")
    assert look("AMD Instinct MI355X", "gfx950", (256, 256, 256)) == (v[2], 1)


def test_wisdom_selection_board_cu_count(tmp_path):
    """Boards of one architecture can report the same device name (every
    gfx950 board here reports "AMD Radeon Graphics"); a record's compute-unit
    count tells them apart at levels 1 and 2, and a record or caller that
    states none matches any board of that name."""
    v = [kl.kl_variant_name(kl.ADVEC_U, kl.F32, i) for i in range(1, 4)]
    d = str(tmp_path)
    name = "AMD Radeon Graphics"
    (tmp_path / "advec_u.wisdom").write_text("\n".join([
        _rec(v[0], (256, 256, 256), device=name, cu=256),
        _rec(v[1], (256, 256, 256), device=name, cu=304),
    ]) + "\n")
    look = lambda cu, size=(256, 256, 256): kl.kl_wisdom_lookup(d, kl.ADVEC_U, kl.F32, name, "gfx950", *size,
                                                                 cu_count=cu)
    assert look(256) == (v[0], 1)
    assert look(304) == (v[1], 1)
    # another board of the same name and architecture: level 3 (same architecture)
    assert look(128) == (v[1], 3)
    assert look(256, (300, 300, 300)) == (v[0], 2)
    # no count given: any board of that name, the later record wins the tie
    assert look(0) == (v[1], 1)
    # a record without a count matches every board of its name
    with open(tmp_path / "advec_u.wisdom", "a") as f:
        f.write(_rec(v[2], (256, 256, 256), device=name) + "\n")
    assert look(128) == (v[2], 1)


def test_wisdom_other_kernel_records_ignored(tmp_path):
    v1 = kl.kl_variant_name(kl.DIFF_UVW, kl.F32, 1)
    (tmp_path / "advec_u.wisdom").write_text(_rec(v1, (64, 64, 64), kernel="diff_uvw") + "\n")
    assert kl.kl_wisdom_lookup(str(tmp_path), kl.ADVEC_U, kl.F32, "AMD Instinct MI355X", "gfx950",
                               64, 64, 64) == ("default", 5)


def test_committed_wisdom_names_registered_configurations():
    """Every record of the committed wisdom files names a configuration this
    build has (a record naming a missing one would be skipped at selection,
    so a stale record would silently fall back to another choice)."""
    kernels = {name: k for k, name in kl.KERNEL_NAMES.items()}
    dtypes = {"f32": kl.F32, "f64": kl.F64}
    wdir = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "wisdom")
    names = {}
    seen = 0
    for fn in sorted(os.listdir(wdir)):
        with open(os.path.join(wdir, fn)) as f:
            for line in f:
                if not line.strip():
                    continue
                rec = json.loads(line)
                batch = rec["kernel"] == "advec_diff_batch"  # batch-level records (kl_batch_tune)
                key = (kl.ADVEC_DIFF if batch else kernels[rec["kernel"]], dtypes[rec["dtype"]])
                if key not in names:
                    names[key] = {kl.kl_variant_name(*key, i) for i in range(kl.kl_num_variants(*key))}
                ok = rec["variant"] in names[key] or (batch and rec["variant"] == "per_grid")
                assert ok, f"{fn}: {rec['variant']} ({rec['dtype']}) is not registered"
                assert rec["kernel"] + ".wisdom" == fn
                seen += 1
    assert seen > 0
