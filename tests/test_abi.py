"""The C-ABI library: builds for gfx950, loads, and exports every symbol the
header declares (no compute calls: those need a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "imexds.h")
HDR_EU = os.path.join(ROOT, "include", "imexds_euler.h")
HDR_CR = os.path.join(ROOT, "include", "imexds_creation.h")
HDR_CT = os.path.join(ROOT, "include", "imexds_ctube.h")
LIB = os.path.join(ROOT, "paper_2211_00705_amd", "libimexds.so")


def declared(hdr=HDR):
    txt = open(hdr).read()
    return sorted(set(re.findall(r"\b(imexds_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    d = declared()
    for name in ("imexds_create", "imexds_set_state", "imexds_step", "imexds_run",
                 "imexds_get_state", "imexds_destroy", "imexds_strerror"):
        assert name in d
    d = declared(HDR_EU)
    for name in ("imexds_eu_create", "imexds_eu_set_state", "imexds_eu_step", "imexds_eu_run",
                 "imexds_eu_get_state", "imexds_eu_get_problems", "imexds_eu_destroy"):
        assert name in d
    assert not set(d) & set(declared())
    assert declared(HDR_CR) == ["imexds_creation_rp", "imexds_creation_rp_noalloc"]
    d = declared(HDR_CT)
    for name in ("imexds_ct_create", "imexds_ct_set_state", "imexds_ct_step", "imexds_ct_run",
                 "imexds_ct_get_state", "imexds_ct_get_problems", "imexds_ct_destroy"):
        assert name in d
    assert not set(d) & (set(declared()) | set(declared(HDR_EU)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    syms = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared() + declared(HDR_EU) + declared(HDR_CR) + declared(HDR_CT)
               if n not in syms]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_maps_every_symbol():
    from paper_2211_00705_amd import imexds
    assert sorted(imexds.EXPORTED) == declared()
    assert imexds.imexds_strerror(-1) == "invalid argument"
    assert imexds.imexds_strerror(0) == "ok"
    from paper_2211_00705_amd import euler
    assert sorted(euler.EXPORTED) == declared(HDR_EU)
    from paper_2211_00705_amd import creation
    assert sorted(creation.EXPORTED) == declared(HDR_CR)
    from paper_2211_00705_amd import ctube
    assert sorted(ctube.EXPORTED) == declared(HDR_CT)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_contains_gfx950_code():
    # the offload bundle of the library built here names its target
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
