"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the host-only partition count and argument validation
behave as documented (no device calls)."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2605_16564_amd import native as N
from paper_2605_16564_amd import synth
from oracle import oracle as O

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib():
    if not N.LIB_PATH.exists():
        from paper_2605_16564_amd import build
        build.build()
    return N.lib()


def test_exports_match_header(lib):
    header = (ROOT / "include" / "pam.h").read_text()
    declared = set(re.findall(r"\b(pam_[a-z_]+)\s*\(", header))
    assert declared == set(N.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def test_struct_sizes_match_header(tmp_path):
    names = ["pam_grid", "pam_dict", "pam_samples", "pam_enet_opts", "pam_fit_stats",
             "pam_refine_opts", "pam_field", "pam_select_opts", "pam_darcy_opts"]
    src = tmp_path / "sz.c"
    fmt = " ".join(["%zu"] * len(names))
    args = ",".join(f"sizeof({n})" for n in names)
    src.write_text('#include <stdio.h>\n#include "pam.h"\nint main(){printf("' + fmt + '\\n",'
                   + args + ');}\n')
    import subprocess
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", str(ROOT / "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(s) for s in (N.PamGrid, N.PamDict, N.PamSamples, N.PamEnetOpts,
                                  N.PamFitStats, N.PamRefineOpts, N.PamField, N.PamSelectOpts,
                                  N.PamDarcyOpts)]
    assert got == want


@pytest.mark.parametrize("make", [lambda: synth.circle64(), lambda: synth.facies256(n_sub=8),
                                  lambda: synth.layered3d(nx=12, ny=10, nz=17, sub=(2, 2, 3)),
                                  lambda: synth.disc_field(5003), lambda: synth.step1d(64)])
def test_partition_count_matches_oracle(lib, make):
    from paper_2605_16564_amd import api
    g = make()
    off, nmax = api.partition_count(g)
    S = O.partition(g)
    assert np.array_equal(off, S["off"])
    assert nmax == int(np.diff(S["off"]).max())


def test_bad_grid_rejected(lib):
    from paper_2605_16564_amd import api
    g = synth.circle64()
    g.breaks = [np.array([0, 40, 30, 64], np.int32), g.breaks[1], g.breaks[2]]
    g.n_sub = [3, 2, 1]
    with pytest.raises(N.PamError, match="increase"):
        api.partition_count(g)
    g = synth.circle64()
    g.overlap = -0.5
    with pytest.raises(N.PamError, match="overlap"):
        api.partition_count(g)
    g = synth.circle64()
    g.dim = 4
    with pytest.raises(N.PamError):
        api.partition_count(g)
