"""The C-ABI library loads and exports every function include/ibmc.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibmc_[a-z_0-9]+)\s*\(", text)))


def test_header_lists_the_boundary():
    names = declared_functions()
    for must in ("ibmc_load_mlp", "ibmc_check_property", "ibmc_coverage", "ibmc_check_batch",
                 "ibmc_proposer_train", "ibmc_check_property_ranked", "ibmc_replay", "ibmc_decode_point"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1907_12933_amd import ibmc
    lib = ibmc.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding describes exactly these functions
    assert sorted(ibmc.SIGNATURES) == declared_functions()


def test_struct_sizes_match_header_layout(tmp_path):
    # compile a probe against the header with the host C compiler and compare
    # every struct size and a few field offsets with the ctypes mirror
    from paper_1907_12933_amd import ibmc
    import subprocess
    probe = tmp_path / "probe.c"
    structs = ["ibmc_mlp_desc", "ibmc_check_opts", "ibmc_cex", "ibmc_check_summary", "ibmc_property",
               "ibmc_ball_property", "ibmc_cov_params", "ibmc_cov_summary", "ibmc_train_opts"]
    body = "\n".join(f'printf("{s} %zu\\n", sizeof({s}));' for s in structs)
    body += '\nprintf("off_points %zu\\n", offsetof(ibmc_check_summary, points));'
    body += '\nprintf("off_seconds %zu\\n", offsetof(ibmc_check_summary, seconds));'
    body += '\nprintf("off_rank %zu\\n", offsetof(ibmc_cex, rank));'
    probe.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ibmc.h"\nint main(void){' + body + 'return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for s in structs:
        assert int(out[s]) == ctypes.sizeof(getattr(ibmc, s)), s
    assert int(out["off_points"]) == ibmc.ibmc_check_summary.points.offset
    assert int(out["off_seconds"]) == ibmc.ibmc_check_summary.seconds.offset
    assert int(out["off_rank"]) == ibmc.ibmc_cex.rank.offset


def test_host_decode_matches_oracle(orc):
    # ibmc_decode_point is host code (no device): it must agree with the
    # oracle's own decoder on every rank of small domains
    from paper_1907_12933_amd import ibmc
    for n, m, k in [(7, 3, 2), (9, 2, 3), (6, 4, 1), (8, 2, 4)]:
        for rank in range(orc.points(n, m, k)):
            p1, d1 = ibmc.ibmc_decode_point(n, m, k, rank)
            p2, d2 = orc.decode(n, m, k, rank)
            assert list(p1) == list(p2) and list(d1) == list(d2)
    with pytest.raises(ibmc.IbmcError):
        ibmc.ibmc_decode_point(7, 3, 2, orc.points(7, 3, 2))
