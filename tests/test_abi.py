"""The C ABI library loads and exports every symbol include/sbx.h declares;
host-only entry points work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sbx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sbx_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1210_1736_amd import sbx
    lib = ctypes.CDLL(sbx.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_validate_hierarchies_host_only():
    from paper_1210_1736_amd import sbx
    ok = sbx.make_hierarchy([(128, 1.0, 0.25), (128, 4.0, 0.25), (128, 20.0, 1.0)], sbx.SBX_CENTRE_COM)
    assert sbx.sbx_validate_hierarchies([ok]) == sbx.SBX_OK
    assert sbx.sbx_q_crit(128, 1.0, 4.0, 20.0) == pytest.approx(0.25)
    assert sbx.sbx_q_crit(64, 3.5, 28.0, 105.0) == pytest.approx(0.25)
    low = sbx.make_hierarchy([(128, 1.0, 0.2), (128, 4.0, 0.2), (128, 20.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([low]) == sbx.SBX_EQCRIT
    nonest = sbx.make_hierarchy([(128, 5.0, 1.0), (128, 4.0, 1.0), (128, 20.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([nonest]) == sbx.SBX_EINVAL
    mixedN = sbx.make_hierarchy([(64, 1.0, 1.0), (128, 4.0, 1.0), (128, 20.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([mixedN]) == sbx.SBX_EINVAL
    sat_flat = sbx.make_hierarchy([(128, 1.0, 0.5), (128, 6.0, 0.5), (128, 20.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([ok, sat_flat]) == sbx.SBX_EINVAL
    sat = sbx.make_hierarchy([(128, 1.0, 1.0), (128, 6.0, 1.0), (128, 20.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([ok, sat]) == sbx.SBX_OK
    other_outer = sbx.make_hierarchy([(128, 1.0, 1.0), (128, 6.0, 1.0), (128, 30.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([ok, other_outer]) == sbx.SBX_EINVAL
    single_com = sbx.make_hierarchy([(64, 5.0, 1.0)], sbx.SBX_CENTRE_COM)
    assert sbx.sbx_validate_hierarchies([single_com]) == sbx.SBX_EINVAL
    odd = sbx.make_hierarchy([(96, 5.0, 1.0)])
    assert sbx.sbx_validate_hierarchies([odd]) == sbx.SBX_EINVAL


def test_library_agrees_with_oracle_on_qcrit_table():
    """Host geometry of the library and the oracle's Eq. 9 on the Table 3 set-up."""
    from paper_1210_1736_amd import sbx
    from oracle import pm_oracle as O
    for N in (64, 128, 256):
        assert sbx.sbx_q_crit(N, 3.5, 28.0, 105.0) == O.q_crit(N, 3.5, 28.0, 105.0)


def test_fft_schedule_pin_host_only():
    """sbx_set_fft_schedule takes 0, 16 or 32 and rejects anything else (host
    state only: no device call)."""
    from paper_1210_1736_amd import sbx
    for v in (16, 32, 0):
        sbx.sbx_set_fft_schedule(v)
    for bad in (-1, 8, 24, 64):
        with pytest.raises(sbx.SbxError):
            sbx.sbx_set_fft_schedule(bad)
    sbx.sbx_set_fft_schedule(0)


def test_fft_form_pin_host_only():
    """sbx_set_fft_form takes 0, 3 or 5 and rejects anything else (host
    state only: no device call)."""
    from paper_1210_1736_amd import sbx
    for f in (3, 5, 0):
        sbx.sbx_set_fft_form(f)
    for bad in (-1, 1, 4, 6):
        with pytest.raises(sbx.SbxError):
            sbx.sbx_set_fft_form(bad)
    sbx.sbx_set_fft_form(0)


def test_plane_threads_pin_host_only():
    """sbx_set_plane_threads takes 0, 256, 512 or 1024 and rejects anything
    else with SBX_EINVAL (host state only: no device call)."""
    from paper_1210_1736_amd import sbx
    for nt in (256, 512, 1024, 0):
        sbx.sbx_set_plane_threads(nt)
    for bad in (-1, 64, 128, 300, 2048):
        with pytest.raises(sbx.SbxError) as e:
            sbx.sbx_set_plane_threads(bad)
        assert e.value.status == sbx.SBX_EINVAL
    sbx.sbx_set_plane_threads(0)
