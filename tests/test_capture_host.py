"""Capture files on the host (no GPU): the C header reader and the Python
array reader agree with a file written to the documented format, and
malformed files are refused."""
import json

import numpy as np
import pytest

from paper_2303_12374_amd import kl


def write_capture(path, dtype=np.float32):
    hdr = {"kernel": "advec_u", "kernel_id": 0, "dtype": "f32" if dtype == np.float32 else "f64",
           "problem_size": [4, 3, 2], "gc": 1, "off": 31, "jstride": 32, "kstride": 160, "dxi": 4.0,
           "dyi": 3.0, "bc": 0, "visc": 0.0, "dt": 0.0,
           "arrays": [{"name": "dzi", "elems": 4}, {"name": "dzhi", "elems": 4}]
           + [{"name": n, "elems": 700} for n in ("u", "v", "w", "ut")]}
    rng = np.random.default_rng(0)
    arrays = {a["name"]: rng.standard_normal(a["elems"]).astype(dtype) for a in hdr["arrays"]}
    with open(path, "wb") as f:
        f.write(b"KLCAP 1\n" + json.dumps(hdr).encode() + b"\n")
        for a in hdr["arrays"]:
            f.write(arrays[a["name"]].tobytes())
    return hdr, arrays


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_capture_header_and_arrays_round_trip(tmp_path, dtype):
    p = tmp_path / "x.klcap"
    hdr, arrays = write_capture(p, dtype)
    assert kl.kl_capture_info(p) == hdr
    h2, a2 = kl.read_capture(p)
    assert h2 == hdr
    for name, arr in arrays.items():
        assert np.array_equal(a2[name], arr)


def test_malformed_captures_are_refused(tmp_path):
    bad = tmp_path / "bad.klcap"
    bad.write_bytes(b"NOTCAP\n{}\n")
    with pytest.raises(kl.KLError) as e:
        kl.kl_capture_info(bad)
    assert e.value.code == kl.ERR_INVALID
    bad.write_bytes(b"KLCAP 1\n{not json\n")
    with pytest.raises(kl.KLError):
        kl.kl_capture_info(bad)
    with pytest.raises(kl.KLError) as e:
        kl.kl_capture_info(tmp_path / "missing.klcap")
    assert e.value.code == kl.ERR_IO


def test_capture_switch_needs_no_device(tmp_path):
    kl.kl_set_capture("advec_u,diff_smag", tmp_path)
    kl.kl_set_capture(None)
