"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/pf.h declares, and validates configurations."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


@pytest.fixture(scope="module")
def pf():
    from paper_1212_1639_amd import pf as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1212_1639_amd import build
        build.build()
    return mod


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pf_[a-z_]+)\s*\(", text,
                                 re.M)))


def test_header_declarations_match_binding(pf):
    assert declared_symbols() == sorted(pf.EXPORTS)


def test_library_exports_every_declared_symbol(pf):
    out = subprocess.run(["nm", "-D", "--defined-only", pf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pf_[a-z_]+)$", out, re.M))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(pf.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_fields(pf):
    assert [pf.lib().pf_fields(m) for m in range(4)] == [1, 5, 1, 6]
    assert pf.lib().pf_fields(9) == 0


def test_workspace_bytes_and_validation(pf):
    good = pf.make_config("ll_pl", 1 << 20, 1, scheme=pf.STRATIFIED, a_v=2, b_v=1, a_w=2, b_w=1,
                          x0_var=10)
    nb = pf.workspace_bytes(good)
    # records (2 x 5 fields x 4 B) and CDF (2 x 4 B) per particle
    assert (1 << 20) * (40 + 8) <= nb < (1 << 20) * 52
    keep = pf.make_config("ll_pl", 1 << 20, 1, scheme=pf.STRATIFIED, a_v=2, b_v=1, a_w=2, b_w=1,
                          x0_var=10, flags=pf.FLAG_KEEP_ANCESTORS)
    assert pf.workspace_bytes(keep) >= nb + 4 * (1 << 20)  # plus the ancestors
    bad = [
        dict(n=0), dict(n=1 << 31), dict(scheme=7), dict(scheme=4), dict(precision=3),
        dict(strategy=9),
        dict(items_per_thread=3), dict(x0_var=-1.0), dict(a_v=0.5), dict(flags=8),
    ]
    for b in bad:
        kw = dict(model="ll_pl", n=1024, seed=1, scheme=pf.STRATIFIED, a_v=2, b_v=1, a_w=2, b_w=1,
                  x0_var=10)
        kw.update(b)
        cfg = pf.make_config(kw.pop("model"), kw.pop("n"), kw.pop("seed"), **kw)
        with pytest.raises(pf.PFError):
            pf.workspace_bytes(cfg)
    # above one LDS window the cut-point table lives in the workspace (one
    # int32 per particle) and is built from the tile scan, so the look-back
    # scan is refused with it
    small = pf.make_config("ll_pf", 2048, 1, strategy=pf.SEARCH_CUTPOINT, items_per_thread=4,
                           sigma_v2=1, sigma_w2=0.1, x0_var=10)
    big = pf.make_config("ll_pf", 1 << 16, 1, strategy=pf.SEARCH_CUTPOINT, items_per_thread=4,
                         sigma_v2=1, sigma_w2=0.1, x0_var=10)
    binary = pf.make_config("ll_pf", 1 << 16, 1, strategy=pf.SEARCH_BINARY, items_per_thread=4,
                            sigma_v2=1, sigma_w2=0.1, x0_var=10)
    assert pf.workspace_bytes(small) > 0
    assert pf.workspace_bytes(big) >= pf.workspace_bytes(binary) + 4 * (1 << 16)
    cfg = pf.make_config("ll_pf", 1 << 16, 1, strategy=pf.SEARCH_CUTPOINT, sigma_v2=1,
                         sigma_w2=0.1, x0_var=10, flags=pf.FLAG_LOOKBACK_SCAN)
    with pytest.raises(pf.PFError, match="cut-point"):
        pf.workspace_bytes(cfg)
    # merge needs sorted uniforms once the CDF exceeds a window
    cfg = pf.make_config("ll_pf", 1 << 16, 1, scheme=pf.MULTINOMIAL, strategy=pf.SEARCH_MERGE,
                         sigma_v2=1, sigma_w2=0.1, x0_var=10)
    with pytest.raises(pf.PFError, match="sorted"):
        pf.workspace_bytes(cfg)
    # double-precision SV-PL at 4 items per thread is switched off; the
    # default tile size for it is 1 item per thread
    svp = dict(x0_mean=-1.0, x0_var=0.1, prior_mean=[-0.05, 0.95], prior_prec=[1.0, 0.0, 1.0],
               a_s=2.0, d_s=0.04)
    off = pf.make_config("sv_pl", 1 << 14, 1, scheme=pf.SYSTEMATIC, precision=pf.FP64,
                         items_per_thread=4, **svp)
    with pytest.raises(pf.PFError, match="switched off"):
        pf.workspace_bytes(off)
    for ipt in (0, 1, 2, 8):
        ok = pf.make_config("sv_pl", 1 << 14, 1, scheme=pf.SYSTEMATIC, precision=pf.FP64,
                            items_per_thread=ipt, **svp)
        assert pf.workspace_bytes(ok) > 0
    f32 = pf.make_config("sv_pl", 1 << 14, 1, scheme=pf.SYSTEMATIC, precision=pf.FP32,
                         items_per_thread=4, **svp)
    assert pf.workspace_bytes(f32) > 0
    # sorted multinomial: accepted in FP64 at any tile size and in FP32 at 1,
    # 2 and 8 items per thread, never with the look-back scan
    sm = pf.make_config("ll_pf", 1 << 16, 1, scheme=pf.SORTED_MULTINOMIAL, sigma_v2=1,
                        sigma_w2=0.1, x0_var=10)
    assert pf.workspace_bytes(sm) > 0
    for ipt, ok in ((0, True), (2, True), (4, False)):
        s32 = pf.make_config("ll_pf", 1 << 16, 1, scheme=pf.SORTED_MULTINOMIAL, precision=pf.FP32,
                             items_per_thread=ipt, sigma_v2=1, sigma_w2=0.1, x0_var=10)
        if ok:
            assert pf.workspace_bytes(s32) > 0
        else:
            with pytest.raises(pf.PFError, match="sorted multinomial"):
                pf.workspace_bytes(s32)
    sm.flags = pf.FLAG_LOOKBACK_SCAN
    with pytest.raises(pf.PFError, match="tile scan"):
        pf.workspace_bytes(sm)
    cfg = pf.make_config("sv_pl", 100, 1, prior_prec=[1.0, 2.0, 1.0], a_s=2, d_s=0.04, x0_var=1)
    with pytest.raises(pf.PFError, match="positive definite"):
        pf.workspace_bytes(cfg)


def test_checkpoint_calls_without_a_filter(pf):
    # the snapshot size of no filter is 0; save and restore refuse NULL
    L = pf.lib()
    assert L.pf_checkpoint_bytes(None) == 0
    buf = (ctypes.c_uint8 * 64)()
    assert L.pf_checkpoint_save(None, buf, 64) == pf.EINVAL
    assert L.pf_checkpoint_restore(None, buf, 64) == pf.EINVAL
