"""Capture and replay on the GPU: a captured launch holds exactly the data
the kernel read (bitwise), replaying it on that data reproduces the
launch's output bitwise, only the first launch per problem size is
captured, and tuning from a capture writes a wisdom record that the
selection then uses."""
import glob
import os

import numpy as np
import pytest
import torch

from paper_2303_12374_amd import inputs

pytestmark = pytest.mark.gpu


def kl():
    from paper_2303_12374_amd import kl as m
    return m


@pytest.fixture(autouse=True)
def scratch_wisdom(tmp_path):
    m = kl()
    m.kl_set_wisdom_dir(str(tmp_path / "wisdom"))
    yield
    m.kl_set_capture(None)
    m.kl_set_wisdom_dir(None)


def make_state(m, shape, dtype, gc, seed):
    g = m.Grid(*shape, dtype=dtype, gc=gc)
    npd = m.NP_DTYPE[dtype]
    fs = [f.astype(npd) for f in inputs.random_fields(seed, *shape)]
    dev = [g.upload(f) for f in fs]
    m.kl_fill_ghosts(g, *dev)
    rng = np.random.default_rng(seed)
    tend = [g.upload(rng.uniform(-1, 1, (shape[2], shape[1], shape[0])).astype(npd), fill=0.0) for _ in range(3)]
    ev = g.upload(inputs.evisc_field(seed, *shape).astype(npd))
    m.kl_fill_scalar(g, ev)
    return g, dev, tend, ev


def replay(m, hdr, arrays, kernel):
    """Run the default configuration on the captured data; returns the
    tendency outputs (host)."""
    dtype = m.F32 if hdr["dtype"] == "f32" else m.F64
    itot, jtot, ktot = hdr["problem_size"]
    elems = len(arrays["u"])
    g = m.Grid(itot, jtot, ktot, dtype=dtype, bc=hdr["bc"], gc=hdr["gc"],
               layout=(hdr["off"], hdr["jstride"], hdr["kstride"], elems + 64))
    g.dzi.copy_(torch.from_numpy(arrays["dzi"]))
    g.dzhi.copy_(torch.from_numpy(arrays["dzhi"]))
    names = ["u", "v", "w", "ut", "vt", "wt", "evisc"]
    bufs = {}
    for n in names:
        if n in arrays:
            t = g.full(0.0)
            t[:elems].copy_(torch.from_numpy(arrays[n]))
            bufs[n] = t
    nout = 1 if kernel in (m.ADVEC_U, m.ADVEC_U_2I5) else 3
    fields = [bufs["u"], bufs["v"], bufs["w"]] + [bufs.get(n, g.full(0.0)) for n in ("ut", "vt", "wt")]
    if kernel == m.DIFF_SMAG:
        fields.append(bufs["evisc"])
    m.kl_launch_variant(g, kernel, 0, fields, hdr["visc"])
    return g, [fields[3 + q] for q in range(nout)]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_capture_holds_the_launch_and_replays_bitwise(tmp_path, dtype):
    m = kl()
    cdir = tmp_path / "cap"
    m.kl_set_capture("advec_u,diff_uvw,diff_smag", cdir)
    shape = (40, 24, 12)
    g1, dev1, tend1, _ = make_state(m, shape, dtype, 1, 3)
    g3, dev3, tend3, ev3 = make_state(m, shape, dtype, 3, 4)
    before = {"advec_u": tend1[0].clone(), "diff_smag": [t.clone() for t in tend3]}
    m.kl_advec_u(g1, tend1[0], *dev1)
    m.kl_diff_smag(g3, *tend3, *dev3, ev3)
    m.kl_advec_u(g1, tend1[0], *dev1)          # same size again: not captured twice
    torch.cuda.synchronize()
    files = sorted(glob.glob(str(cdir / "*.klcap")))
    d = "f32" if dtype == 0 else "f64"
    assert [os.path.basename(f) for f in files] == [f"advec_u_{d}_40x24x12.klcap", f"diff_smag_{d}_40x24x12.klcap"]

    # the advec_u capture: the fields as launched (ut before the launch)
    hdr, arrays = m.read_capture(files[0])
    assert hdr["kernel"] == "advec_u" and hdr["problem_size"] == list(shape) and hdr["gc"] == 1
    base = g1.off - hdr["off"]
    n = len(arrays["u"])
    for name, t in (("u", dev1[0]), ("v", dev1[1]), ("w", dev1[2]), ("ut", before["advec_u"])):
        got = t[base:base + n].cpu().numpy()
        assert np.array_equal(got, arrays[name], equal_nan=True), f"captured {name} differs"
    assert np.array_equal(arrays["dzi"], g1.dzi.cpu().numpy())
    assert m.kl_capture_info(files[0]) == hdr

    # replaying the diff_smag capture reproduces the launch's outputs bitwise
    hdr3, arrays3 = m.read_capture(files[1])
    g, outs = replay(m, hdr3, arrays3, m.DIFF_SMAG)
    for q in range(3):
        want = g3.interior(tend3[q]).cpu().numpy()
        assert np.array_equal(g.interior(outs[q]).cpu().numpy(), want), f"replayed tendency {q} differs"


def test_tuning_from_a_capture_writes_a_selected_record(tmp_path):
    m = kl()
    cdir, wdir = tmp_path / "cap", tmp_path / "wis"
    m.kl_set_capture("advec_u_2i5", cdir)
    shape = (128, 64, 32)
    g, dev, tend, _ = make_state(m, shape, 0, 3, 5)
    m.kl_advec_u_2i5(g, tend[0], *dev)
    torch.cuda.synchronize()
    m.kl_set_capture(None)
    path = str(cdir / "advec_u_2i5_f32_128x64x32.klcap")
    res = m.kl_tune_capture(path, wdir, budget_s=30.0)
    assert len(res) >= 2 and all(ms > 0 for _, ms in res), "a configuration failed the bitwise check"
    lines = open(wdir / "advec_u_2i5.wisdom").read().strip().splitlines()
    assert len(lines) == 1 and '"problem_size":[128,64,32]' in lines[0]
    best = min(res, key=lambda r: r[1])[0]
    m.kl_set_wisdom_dir(str(wdir))
    assert m.kl_selected_variant(g, m.ADVEC_U_2I5) == best
