"""Planted mistakes in copies of the oracle must each fail at least one pin.

Each mutant is a small textual edit of oracle/pdc_oracle.c (a dropped
term, a flipped sign or comparison, a transposed index, the wrong rounding or
median rank), compiled with the oracle's own flags into a temporary directory.
The pins in tests/pins.py are then run against it; the test passes when some
pin rejects the mutant.  CPU only; the committed oracle is never modified.
"""
import os
import subprocess

import pytest

from oracle import oracle
from tests import pins

MUTANTS = [
    ("drop 14-bit mask", "(float)(raw[p] & 0x3FFF)", "(float)(raw[p])"),
    ("dark added", "float t = a - dark[p];", "float t = a + dark[p];"),
    ("dark sign flipped", "float t = a - dark[p];", "float t = dark[p] - a;"),
    ("gain multiplied", "frames1[p] = t * k;", "frames1[p] = t * gain[p];"),
    ("gain ignored", "frames1[p] = t * k;", "frames1[p] = t;"),
    ("upper median", "tmp[(B - 1) / 2]", "tmp[B / 2]"),
    ("median off by one", "tmp[(B - 1) / 2]", "tmp[(B - 1) / 2 + 1]"),
    ("median over whole row", "memcpy(tmp, row, sizeof(float) * (size_t)B);",
     "memcpy(tmp, frames1 + ((int64_t)t * H + r) * W, sizeof(float) * (size_t)B);"),
    ("common mode added", "frames2[p] = frames1[p] - med[", "frames2[p] = frames1[p] + med["),
    ("wrong bank of pixel", "med[((int64_t)t * H + r) * nb + c / B]", "med[((int64_t)t * H + r) * nb + c % nb]"),
    ("seed >=", "if (!(vp > t_seed)) continue;", "if (!(vp >= t_seed)) continue;"),
    ("tie-break reversed", "(vp == vq && p < q)", "(vp == vq && p > q)"),
    ("ties always win", "(vp == vq && p < q)", "(vp == vq)"),
    ("window crosses tiles", "if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;\n                        int64_t q",
     "if (cc < 0 || cc >= W) continue;\n                        if ((int64_t)t * H + rr < 0 || (int64_t)t * H + rr >= (int64_t)T * H) continue;\n                        int64_t q"),
    ("sum skips centre", "float vj = v[((int64_t)t * H + rr) * W + cc];",
     "if (rr == r && cc == c) continue;\n                        float vj = v[((int64_t)t * H + rr) * W + cc];"),
    ("neighbour mask >=", "(vj > t_nb ? vj : 0.0f)", "(vj >= t_nb ? vj : 0.0f)"),
    ("neighbour mask dropped", "(vj > t_nb ? vj : 0.0f)", "vj"),
    ("sum transposed index", "float vj = v[((int64_t)t * H + rr) * W + cc];",
     "float vj = v[((int64_t)t * H + (rr < W && cc < H ? cc : rr)) * W + (rr < W && cc < H ? rr : cc)];"),
    ("sum centre-first order", ["float qsum = 0.0f;",
                                "float vj = v[((int64_t)t * H + rr) * W + cc];"],
     ["float qsum = (vp > t_nb ? vp : 0.0f);",
      "if (rr == r && cc == c) continue;\n                        float vj = v[((int64_t)t * H + rr) * W + cc];"]),
    ("round half away", "(uint32_t)rintf(x)", "(uint32_t)roundf(x)"),
    ("truncate count", "(uint32_t)rintf(x)", "(uint32_t)x"),
    ("thresholds swapped", "float t_seed = n_seed * sigma;", "float t_seed = n_nb * sigma;"),
    ("nb threshold from seed", "float t_nb = n_nb * sigma;", "float t_nb = n_seed * sigma;"),
]


@pytest.fixture(scope="module")
def source():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, name, old, new):
    olds = old if isinstance(old, list) else [old]
    news = new if isinstance(new, list) else [new]
    mutated = source
    for o_, n_ in zip(olds, news):
        assert mutated.count(o_) == 1, "mutation site must be unique: %r" % o_
        mutated = mutated.replace(o_, n_)
    src = tmp_path / "mutant.c"
    src.write_text(mutated)
    lib = str(tmp_path / "libmutant.so")
    oracle.compile_oracle(str(src), lib)
    mut = oracle.load(lib)
    failed = []
    for pin in pins.PINS:
        try:
            pin(mut)
        except AssertionError:
            failed.append(pin.__name__)
            break
        except Exception as e:  # a crash of the mutant also counts as caught
            failed.append("%s (%s)" % (pin.__name__, type(e).__name__))
            break
    assert failed, "mutant '%s' passed every pin" % name
