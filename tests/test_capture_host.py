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


def _write(path, hdr, arrays, cut=0):
    body = b"KLCAP 1\n" + json.dumps(hdr).encode() + b"\n"
    for a in hdr["arrays"]:
        body += arrays[a["name"]][:a["elems"]].tobytes() if a["name"] in arrays else b""
    if cut:
        body = body[:-cut]
    path.write_bytes(body)


def _mut_metric(h, a):
    h["arrays"][0]["elems"] = 3


def _mut_field_short(h, a):
    for x in h["arrays"][2:]:
        x["elems"] = 600  # the ghost box of the header's layout spans 645 cells


def _mut_field_mismatch(h, a):
    h["arrays"][4]["elems"] = 650


def _mut_dtype(h, a):
    h["dtype"] = "f16"


def _mut_kernel_id(h, a):
    h["kernel_id"] = 1  # diff_uvw, but the name says advec_u


def _mut_kernel_range(h, a):
    h["kernel_id"] = 9


def _mut_order(h, a):
    h["arrays"][2], h["arrays"][3] = h["arrays"][3], h["arrays"][2]


def _mut_too_few(h, a):
    del h["arrays"][-1]


def _mut_jstride(h, a):
    h["jstride"] = 5  # < itot + 2


def _mut_off(h, a):
    h["off"] = -1


def _mut_gc_fraction(h, a):
    h["gc"] = 1.5


def _mut_size(h, a):
    h["problem_size"] = [4, 0, 2]


def _mut_size_type(h, a):
    h["problem_size"] = [4, "3", 2]


def _mut_bc(h, a):
    h["bc"] = 7


REFUSALS = [_mut_metric, _mut_field_short, _mut_field_mismatch, _mut_dtype, _mut_kernel_id, _mut_kernel_range,
            _mut_order, _mut_too_few, _mut_jstride, _mut_off, _mut_gc_fraction, _mut_size, _mut_size_type, _mut_bc]


@pytest.mark.parametrize("mutate", REFUSALS, ids=lambda f: f.__name__[5:])
def test_tune_capture_refuses_inconsistent_headers(tmp_path, mutate):
    """A capture whose header disagrees with itself or with the layout it
    describes is refused before any device memory is allocated or any
    kernel runs (this host has no GPU: a device call would fail with
    ERR_DEVICE instead)."""
    p = tmp_path / "x.klcap"
    hdr, arrays = write_capture(p)
    mutate(hdr, arrays)
    _write(p, hdr, arrays)
    with pytest.raises(kl.KLError) as e:
        kl.kl_tune_capture(p, tmp_path / "wisdom", 1.0, stream=0)
    assert e.value.code == kl.ERR_INVALID, kl.kl_last_error()
    assert not (tmp_path / "wisdom").exists()


@pytest.mark.parametrize("cut", [1, 4, 2800])
def test_tune_capture_refuses_truncated_payload(tmp_path, cut):
    p = tmp_path / "x.klcap"
    hdr, arrays = write_capture(p)
    _write(p, hdr, arrays, cut=cut)
    with pytest.raises(kl.KLError) as e:
        kl.kl_tune_capture(p, tmp_path / "wisdom", 1.0, stream=0)
    assert e.value.code == kl.ERR_IO, kl.kl_last_error()
    assert "truncated" in kl.kl_last_error()


def test_tune_capture_accepts_a_consistent_header(tmp_path):
    """The unmodified file passes every check and reaches the device
    upload (which fails on this host without a GPU)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("runs the tuner on a GPU host")
    p = tmp_path / "x.klcap"
    write_capture(p)
    with pytest.raises(kl.KLError) as e:
        kl.kl_tune_capture(p, tmp_path / "wisdom", 1.0, stream=0)
    assert e.value.code == kl.ERR_DEVICE, kl.kl_last_error()
