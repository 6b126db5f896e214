"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a reading
of the paper flipped, a sign or an index changed), builds it with gcc in a
temporary folder, and runs the pins in a child process against that build
(``STEV_ORACLE_LIB``).  The case passes when at least one of the named pins
fails.  Nothing here touches the committed oracle or any GPU code.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stev_oracle.c")

# (name, exact text in stev_oracle.c, replacement, pins expected to catch it)
MUTATIONS = [
    # Eq 8: the ring stores the damped rate rOF q h instead of the undamped q h
    ("ring_stores_damped_rate",
     "ring[j * W + (int)((it - 1) % W)] = q[j] * h;",
     "ring[j * W + (int)((it - 1) % W)] = rOF[j] * q[j] * h;",
     "damped_trajectory"),
    # Eqs 15-16: the low set taken from T_mid up
    ("range_select_swapped",
     "(T < m->T_mid[k]) ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k]",
     "(T >= m->T_mid[k]) ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k]",
     "range_select or thermo"),
    # Eq 10: the high band widened down to bin 3
    ("band_from_bin_3",
     "int k_lo = (W + 3) / 4, k_hi = W / 2;",
     "int k_lo = 3, k_hi = W / 2;",
     "high_band"),
    # Eq 30: (RT / 1 atm)^dN in place of (1 atm / RT)^dN
    ("delta_n_inverted",
     "double K = pow(ORC_PATM / (ORC_R * T), dN) * exp(-dG_RT);\n      double kr = kf / K;\n      double prod_r",
     "double K = pow((ORC_R * T) / ORC_PATM, dN) * exp(-dG_RT);\n      double kr = kf / K;\n      double prod_r",
     "t10_two or t8"),
    # Eq 2: the 90 % rule applied below 1e-20 and the unit value above
    ("eq2_branches_swapped",
     "double ystar = (Y[k] < 1.0e-20) ? 1.0 : 0.9 * Y[k];",
     "double ystar = (Y[k] < 1.0e-20) ? 0.9 * Y[k] : 1.0;",
     "t3"),
    # Eq 13: no cap at 1
    ("rof_uncapped",
     "double r = fmin(rof * rof_star, 1.0);",
     "double r = rof * rof_star;",
     "t7 or damped_trajectory"),
    # Eq 12: rOF update before the ring is full
    ("rof_before_full_ring",
     "if (it >= W) {",
     "if (it >= 1) {",
     "t7 or damped_trajectory"),
]


def _build(src_text, out_dir):
    c = os.path.join(out_dir, "stev_oracle.c")
    with open(c, "w") as f:
        f.write(src_text)
    shutil.copy(os.path.join(ROOT, "oracle", "stev_oracle.h"), out_dir)
    lib = os.path.join(out_dir, "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-o", lib, c, "-lm"])
    return lib


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    lib = _build(text.replace(old, new), str(tmp_path))
    env = dict(os.environ, STEV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (
        f"pins '{pins}' did not catch {name}:\n{r.stdout[-2000:]}")
