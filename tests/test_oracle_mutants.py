"""Planted mistakes in a copy of the oracle source must fail at least one pin.

Each mutant is a small textual change of ``oracle/lbg_oracle.c`` -- a dropped
term, a wrong sign, a wrong index or divisor, a relaxed comparison -- compiled
into a temporary library on the CPU.  The real oracle is never modified.
"""
import os

import pytest

import oracle
from oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "lbg_oracle.c")

MUTANTS = {
    "square_dropped": [("s += d * d;", "s += d;")],
    "tie_to_highest": [("if (d < best) {", "if (d <= best) {")],
    "second_dropped": [("} else if (d < second) {", "} else if (0) {")],
    "split_sign": [("dn = c * (1.0 - eps);", "dn = c * (1.0 + eps);")],
    "split_order": [("C2[(2 * i) * L + l] = store(up", "C2[(2 * i + 1) * L + l] = store(UPX"),
                    ("C2[(2 * i + 1) * L + l] = store(dn", "C2[(2 * i) * L + l] = store(dn"),
                    ("store(UPX", "store(up")],
    "centroid_divisor": [("c0[l] /= (double)M;", "c0[l] /= (double)(M - 1);")],
    "update_divisor": [("sum[k * L + l] / (double)cnt[k]", "sum[k * L + l] / (double)M")],
    "empty_cell_zeroed": [(": C_old[k * L + l];", ": 0.0;")],
    "update_wrong_dim": [("sum[k * L + l] += (double)X[m * L + l];",
                          "sum[k * L + l] += (double)X[m * L];")],
    "distortion_not_mean": [("return s / (double)M;", "return s;")],
    "train_D_not_mean": [("D = s / (double)M;\n      trace_D", "D = s;\n      trace_D")],
    "stop_strict": [("(D_prev - D) <= p->thr * D_prev", "(D_prev - D) < p->thr * D_prev")],
    "stop_first_guard_dropped": [("stop = !first && ", "stop = ")],
    "codebook_stride": [("sqdist(x, C + k * L, L)", "sqdist(x, C + k, L)")],
    "grad_sign": [("gC[(int64_t)idx[m] * L + l] -= s * diff;",
                   "gC[(int64_t)idx[m] * L + l] += s * diff;")],
    "grad_scale": [("double s = 2.0 * g / (double)M;", "double s = g / (double)M;")],
    "fp32_store_ignored": [("return fp32 ? (double)(float)v : v;", "return v;")],
}


def _mutate(text, edits):
    for old, new in edits:
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    return text


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    with open(SRC) as f:
        text = f.read()
    src = tmp_path / f"mut_{name}.c"
    src.write_text(_mutate(text, MUTANTS[name]))
    so = tmp_path / f"libmut_{name}.so"
    oracle.build(src=str(src), out=str(so))
    lib = oracle.load(str(so))
    failed = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except Exception:
            failed.append(pin.__name__)
            break
    assert failed, f"mutant {name} passed every pin"
