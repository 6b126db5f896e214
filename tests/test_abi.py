"""CPU checks of the C ABI: the library loads and exports every symbol the
public header declares, and the parameter/statistics structs match."""

import ctypes as C
import os

import pytest

from paper_1905_09395_amd import stev

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(stev.LIB_PATH):
        from paper_1905_09395_amd import build
        build.build()
    return stev.load()


def test_header_symbols_exported(lib):
    names = stev.header_symbols()
    assert "stev_integrate" in names and "stev_submit" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_default_params(lib):
    p = stev.default_params()
    assert p.precision == stev.F64 and p.thermo == stev.THERMO_POLY
    assert p.ystep_max == 1e-3 and p.delta_max == 1e-2 and p.alpha == 1e-5
    assert p.tol_ring == 0.5 and p.tol_freq == 1e-6 and p.r_fac == 2.0
    assert p.rof_min == 1e-12 and p.dft_window == 13 and p.max_iters == 1000000


def test_struct_sizes_match_header():
    # field order / sizes mirror include/stev.h (checked against a C compile)
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "stev.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(stev_params), sizeof(stev_stats),
         sizeof(stev_mech_desc), sizeof(stev_mlp_cfg), sizeof(stev_mlp_report),
         offsetof(stev_params, max_iters), sizeof(stev_lma_cfg), sizeof(stev_lma_report),
         offsetof(stev_lma_report, train_loss));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = [int(x) for x in out]
    assert sizes == [C.sizeof(stev.Params), C.sizeof(stev.Stats), C.sizeof(stev.MechDesc),
                     C.sizeof(stev.MlpCfg), C.sizeof(stev.MlpReport),
                     stev.Params.max_iters.offset, C.sizeof(stev.LmaCfg),
                     C.sizeof(stev.LmaReport), stev.LmaReport.train_loss.offset]
