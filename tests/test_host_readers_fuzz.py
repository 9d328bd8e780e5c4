"""Malformed inputs to the host-side readers of libkl (no GPU): the JSON
reader behind wisdom selection and the capture-header reader behind
kl_capture_info and kl_tune_capture.  Every input of a bounded, seeded
corpus (truncations, byte changes, deep nesting, odd numbers and escapes,
wrong types) must be parsed or refused with an error code; none may crash.
Run with the address/undefined-behaviour sanitizer build of the host code
(test_host_sanitizers.py) the same corpus also checks memory safety."""
import json
import random

import pytest

from paper_2303_12374_amd import kl

VALID_RECORD = {
    "kernel": "advec_u", "dtype": "f32", "problem_size": [256, 256, 256], "variant": None,
    "params": {"family": 2, "vx": 4, "bx": 64, "by": 4, "kb": 128, "xcd": 3}, "time_ms": 0.123,
    "device": "AMD Radeon Graphics", "arch": "gfx950", "cu_count": 256, "date": "2026-01-01T00:00:00Z",
    "hostname": "h", "hip_runtime": 70000000, "lib_version": "x",
}

ODD_TOKENS = ["1e99999", "-1e-99999", "nan", "Infinity", "-0", "0x10", "1.", ".5", "01", "\"\\u12\"",
              "\"\\ud800\"", "\"\\x41\"", "\"\\", "\"", "{", "}", "[", "]", ":", ",", "true", "fals", "null",
              "\"\x00\"", "9" * 400, "-" * 50, "\"" + "a" * 5000 + "\""]


def corpus(valid: str, seed: int, n: int):
    """Deterministic malformed variants of `valid`."""
    rng = random.Random(seed)
    out = [valid[:k] for k in range(0, len(valid), max(1, len(valid) // 40))]  # truncations
    for _ in range(n):
        s = list(valid)
        kind = rng.randrange(5)
        if kind == 0:  # change bytes
            for _ in range(rng.randrange(1, 4)):
                s[rng.randrange(len(s))] = chr(rng.randrange(1, 128))
        elif kind == 1:  # insert an odd token
            p = rng.randrange(len(s) + 1)
            s[p:p] = list(rng.choice(ODD_TOKENS))
        elif kind == 2:  # delete a span
            a = rng.randrange(len(s))
            del s[a:a + rng.randrange(1, 12)]
        elif kind == 3:  # duplicate a span
            a = rng.randrange(len(s))
            b = min(len(s), a + rng.randrange(1, 30))
            s[a:a] = s[a:b]
        else:  # replace a value by an odd token
            p = valid.find(":", rng.randrange(len(valid)))
            if p >= 0:
                q = p + 1
                while q < len(s) and s[q] not in ",}":
                    q += 1
                s[p + 1:q] = list(rng.choice(ODD_TOKENS))
        out.append("".join(s))
    out += ["[" * 20000 + "]" * 20000, "{\"a\":" * 20000 + "1" + "}" * 20000, "", "\n\n\n", "{}", "[]",
            json.dumps({**json.loads(valid), "problem_size": [1e300, -5, 2 ** 70]}),
            json.dumps({**json.loads(valid), "problem_size": "256"}),
            json.dumps({**json.loads(valid), "device": [1, 2, 3]}),
            json.dumps({**json.loads(valid), "arrays": [{"name": "u", "elems": -1}]}),
            json.dumps({**json.loads(valid), "arrays": [{"name": "u", "elems": 2 ** 62}] * 7})]
    return out


def test_wisdom_reader_survives_malformed_records(tmp_path):
    name = kl.kl_variant_name(kl.ADVEC_U, kl.F32, 1)
    rec = dict(VALID_RECORD, variant=name)
    valid = json.dumps(rec)
    cases = corpus(valid, seed=11, n=400)
    # one file of all cases plus the valid record last: the reader skips what
    # it cannot use and still finds the valid record
    (tmp_path / "advec_u.wisdom").write_text("\n".join(c.replace("\n", " ") for c in cases) + "\n" + valid + "\n")
    got = kl.kl_wisdom_lookup(str(tmp_path), kl.ADVEC_U, kl.F32, "AMD Radeon Graphics", "gfx950", 256, 256, 256,
                              cu_count=256)
    assert got == (name, 1)
    # each case alone: parsed or skipped, never a crash
    for n, c in enumerate(cases[::4]):
        (tmp_path / "advec_u.wisdom").write_text(c.replace("\n", " ") + "\n")
        v, level = kl.kl_wisdom_lookup(str(tmp_path), kl.ADVEC_U, kl.F32, "AMD Radeon Graphics", "gfx950",
                                       256, 256, 256)
        assert level in (1, 2, 3, 4, 5), (n, c[:80])


def _capture_header():
    return {"kernel": "advec_u", "kernel_id": 0, "dtype": "f32", "problem_size": [4, 3, 2], "gc": 1,
            "off": 31, "jstride": 32, "kstride": 160, "dxi": 4.0, "dyi": 3.0, "bc": 0, "visc": 0.0, "dt": 0.0,
            "arrays": [{"name": "dzi", "elems": 4}, {"name": "dzhi", "elems": 4}]
            + [{"name": n, "elems": 700} for n in ("u", "v", "w", "ut")]}


def test_capture_reader_survives_malformed_headers(tmp_path):
    import torch
    valid = json.dumps(_capture_header())
    payload = b"\0" * (4 * (8 + 4 * 700))
    p = tmp_path / "x.klcap"
    for n, c in enumerate(corpus(valid, seed=12, n=300)):
        p.write_bytes(b"KLCAP 1\n" + c.replace("\n", " ").encode("utf-8", "surrogatepass") + b"\n" + payload)
        try:
            kl.kl_capture_info(p)
        except kl.KLError as e:
            assert e.code in (kl.ERR_INVALID, kl.ERR_IO), (n, e)
        except (json.JSONDecodeError, UnicodeDecodeError):
            pass  # the C reader accepted text Python's json does not; the C side did not crash
        if torch.cuda.is_available():
            continue  # on a GPU host an accepted header would start tuning
        try:
            kl.kl_tune_capture(p, tmp_path / "wisdom", 1.0, stream=0)
        except kl.KLError as e:
            # refused on the header, the payload size, or (header accepted) at
            # the first device call of this GPU-less host
            assert e.code in (kl.ERR_INVALID, kl.ERR_IO, kl.ERR_DEVICE), (n, e)
        assert not (tmp_path / "wisdom").exists()
