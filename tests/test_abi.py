"""The C ABI library loads, exports every symbol include/atsne.h declares, and
validates arguments on the host (CPU only: no kernel is launched)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    hdr = (ROOT / "include" / "atsne.h").read_text()
    return sorted(set(re.findall(r"^(?:atsne_status|const char\*)\s+(atsne_\w+)\(", hdr, re.M)))


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ["atsne_knn", "atsne_knn_subset", "atsne_calibrate_p", "atsne_symmetrize", "atsne_symmetrize_csr",
              "atsne_serve_create", "atsne_serve_submit_insert", "atsne_serve_submit_refine", "atsne_serve_wait"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1512_01655_amd import atsne

    L = atsne.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(atsne.EXPORTS) == _declared()


def test_host_side_validation():
    from paper_1512_01655_amd import atsne

    L = atsne.load()
    b = ctypes.c_size_t()
    # sizes and ranges are checked before anything touches a device
    assert L.atsne_knn_workspace_size(10, 10, 4, 0, 10, 0, ctypes.byref(b)) == atsne.E_K_RANGE
    assert L.atsne_knn_workspace_size(10, 10, 4, 0, 3, 2, ctypes.byref(b)) == atsne.E_K_RANGE
    assert L.atsne_knn_workspace_size(10, 10, 4, 7, 3, 0, ctypes.byref(b)) == atsne.E_INVALID_ARG
    assert L.atsne_knn_workspace_size(1, 1, 4, 0, 1, 0, ctypes.byref(b)) == atsne.E_INVALID_ARG
    assert L.atsne_knn_workspace_size(70000, 70000, 784, 0, 90, 0, ctypes.byref(b)) == atsne.OK
    assert b.value > 70000 * 784 * 4
    assert L.atsne_knn(None, 10, 4, 4, 0, 3, 0, None, None, None, None, None, 0, None) == atsne.E_INVALID_ARG
    assert L.atsne_calibrate_p(None, None, 10, 30, 10.0, 0.0, 0, 0, None, None, None, None, None) == \
        atsne.E_INVALID_ARG
    assert L.atsne_symmetrize_workspace_size(100, 900, ctypes.byref(b)) == atsne.OK
    assert L.atsne_serve_create(None, None, 0, 0, 30.0, None) == atsne.E_INVALID_ARG
    assert b"bad arguments" in L.atsne_last_error()
    # attractive forces: empty input is a no-op; checks precede any launch
    assert L.atsne_attractive_forces(None, None, None, 0, 0, None, 2, None, 1.0, 1.0, 0, 1.0, None, None) == atsne.OK
    assert L.atsne_attractive_forces(None, None, None, 5, 0, None, 2, None, 1.0, 1.0, 0, 1.0, None,
                                     None) == atsne.E_INVALID_ARG
    fake = ctypes.c_void_p(16)  # never dereferenced: the call fails before use
    assert L.atsne_attractive_forces(fake, fake, fake, 5, 9, fake, 4, None, 1.0, 1.0, 0, 1.0, fake,
                                     None) == atsne.E_UNSUPPORTED
    assert L.atsne_attractive_forces(fake, fake, fake, 5, 9, fake, 2, fake, 4.0, 0.0, 0, 1.0, fake,
                                     None) == atsne.E_INVALID_ARG


@pytest.mark.parametrize("prec,k,kc", [(0, 90, 0), (1, 90, 0), (2, 150, 0), (0, 90, 90), (3, 90, 0)])
def test_workspace_grows_with_candidates(prec, k, kc):
    from paper_1512_01655_amd import atsne

    # slots hold at least 768 keys, so the larger candidate count must push
    # k' + 256 + max(k', 128) past that
    small = atsne.knn_workspace_size(20000, 20000, 128, k, ["fp32", "bf16", "fp8", "fp32x3"][prec], kc)
    big = atsne.knn_workspace_size(20000, 20000, 128, k, ["fp32", "bf16", "fp8", "fp32x3"][prec], 4 * k + 50)
    assert big > small > 0
