"""Mutation tests of the oracle's pins: each case plants one plausible
mistake in a copy of oracle/vcaref.c (on the CPU, in a temporary library),
runs the pins of tests/test_oracle.py against it, and requires that at least
one pin fails.  The unmodified source, built the same way, must pass."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vcaref.c")

MUTATIONS = {
    "matrix magnitude off by one": ("78, 75, 73, 70", "78, 75, 74, 70"),
    "cosine fold sign": ("return -kMag[64 - a];", "return kMag[64 - a];"),
    "w-point rows not subsampled": ("c32(k * (32 / w), n)", "c32(k, n)"),
    "horizontal shift off by one": ("int s1 = ilog2(w) + B - 9;", "int s1 = ilog2(w) + B - 8;"),
    "vertical rounding bias dropped": ("floor_div_pow2(acc + ((int64_t)1 << (s2 - 1)), s2)",
                                       "floor_div_pow2(acc, s2)"),
    "truncation instead of floor": ("if (v % d != 0 && v < 0) q -= 1;", ""),
    "output transposed": ("y[i * K + k] = floor_div_pow2", "y[k * K + i] = floor_div_pow2"),
    "weight without the square": ("exp(fabs(r * r - 1.0))", "exp(fabs(r - 1.0))"),
    "DC counted in the energy": ("if (i != 0 || k != 0) e +=", "e +="),
    "signed energy difference in h": ("dh += fabs(Hf[b] - prev[b]);", "dh += Hf[b] - prev[b];"),
    "energy not divided by w^2": ("out[0] = sumH[0] / (cnt[0] * ww);", "out[0] = sumH[0] / cnt[0];"),
    "brightness without the square root": ("sumL[P] += sqrt((double)Df[off + b]);",
                                           "sumL[P] += (double)Df[off + b];"),
}


def build(src_text, out):
    c = out.with_suffix(".c")
    c.write_text(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-I" + os.path.join(ROOT, "oracle"), str(c), "-o", str(out),
                    "-lm"], check=True, capture_output=True)


def pins_pass(lib):
    env = dict(os.environ, VCAREF_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode == 0


def test_unmodified_source_passes(tmp_path):
    lib = tmp_path / "libvcaref_plain.so"
    build(open(SRC).read(), lib)
    assert pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    text = open(SRC).read()
    old, new = MUTATIONS[name]
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    lib = tmp_path / "libvcaref_mut.so"
    build(text.replace(old, new), lib)
    assert not pins_pass(lib), f"no pin catches: {name}"
