"""Mutation check of the oracle's pins (CPU).

Each case plants one plausible mistake in a temporary copy of the oracle's C
source (a dropped term, a wrong sign, an off-by-one window, a transposed
operand, a swapped constant), builds it, and runs the pin suite against it in
a fresh process: the suite must fail. This shows the pins would catch such a
mistake in the real oracle."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sk_oracle.c")

MUTANTS = {
    "decode offset": ("int re = (int)(byte >> 4) - 8;", "int re = (int)(byte >> 4) - 7;"),
    "dropped im term": ("return re * re + im * im;", "return re * re + im;"),
    "square power": ("S2[(f * B + b) * N + i] += p * p;", "S2[(f * B + b) * N + i] += p;"),
    "window off by one": ("for (int64_t bb = b - L + 1; bb <= b; ++bb) {", "for (int64_t bb = b - L; bb <= b; ++bb) {"),
    "history index": ("src = hist + (f * H + (H + bb)) * N;", "src = hist + (f * H + (H + bb + 1 < H ? H + bb + 1 : H - 1)) * N;"),
    "A weight": ("A += (double)S1[idx] / pd;", "A += (double)S1[idx] / (pd * pd);"),
    "Bq weight": ("Bq += (double)S2[idx] / (pd * pd);", "Bq += (double)S2[idx] / pd;"),
    "K factor": ("            V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);",
                 "            V = (Kd - 1.0) / (Kd + 1.0) * (Kd * Bq / (A * A) - 1.0);"),
    "K factor (real-valued path)": ("      else V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);",
                                    "      else V = (Kd + 1.0) / (Kd - 1.0) * (Bq / (A * A) - 1.0);"),
    "real-valued square power": ("          S2[(f * B + b) * N + i] += v * v;", "          S2[(f * B + b) * N + i] += v;"),
    "tilde count": ("            V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)n - 1.0);",
                    "            V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)(n + 1) - 1.0);"),
    "pooled numerator sign": ("__int128 num = (__int128)K * (__int128)R2 - (__int128)R1 * (__int128)R1;", "__int128 num = (__int128)K * (__int128)R2 + (__int128)R1 * (__int128)R1;"),
    "mask ignored": ("if (mask && mask[f * N + i] == 0) continue;", "if (mask && mask[f * N + i] == 2) continue;"),
    "E0 factor inverted": ("e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));", "e0 = ((Kd - 1.0) * (Md + 1.0)) / ((Kd + 1.0) * (Md - 1.0));"),
    "sigma": ("*sigma = sigma_override > 0.0 ? sigma_override : sqrt(4.0 / Kd);", "*sigma = sigma_override > 0.0 ? sigma_override : sqrt(2.0 / Kd);"),
    "flag side": ("if (V > hi) fl |= ORC_FLAG_HIGH;", "if (V >= lo) fl |= ORC_FLAG_HIGH;"),
    "pmf edge": ("double lo = (v == -clip) ? 0.0 : orc_phi(((double)v - 0.5) / sigma);", "double lo = (v == -clip) ? 0.0 : orc_phi(((double)v - 0.4) / sigma);"),
    "n_eff counts zero power": ("if (p <= 0) continue;", "if (p < 0) continue;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    mut = tmp_path / "sk_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", str(mut), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, SK_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"no pin caught the mutant '{name}'"
