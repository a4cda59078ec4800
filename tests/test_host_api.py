"""Host-side checks of the C ABI (no GPU needed): exports, validation, directions, workspace sizes."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2401_08260_amd as ks
from oracle import directions as odir

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "ksum.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ksum_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(ks.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ks.EXPORTED)


def test_status_strings_and_version():
    assert ks.ksum_version().startswith("ksum")
    for st in range(7):
        assert ks.ksum_status_string(st).startswith("KSUM_")


@pytest.mark.parametrize("d,P,seed", [(1, 3, 0), (10, 64, 0), (784, 8, 1), (3072, 2, 3)])
def test_directions_match_oracle_bitwise(d, P, seed):
    assert np.array_equal(ks.ksum_generate_directions(d, P, seed), odir.directions(d, P, seed))


def test_direction_prefix_property():
    a = ks.ksum_generate_directions(50, 256, 2)
    b = ks.ksum_generate_directions(50, 4, 2)
    assert np.array_equal(a[:4], b)


def _st(d, P, kernel, **kw):
    return ks.ksum_check_params(d, P, kernel, ks.make_params(kernel, **kw))


def test_validation_status_codes():
    G, L, N = ks.KSUM_GAUSSIAN, ks.KSUM_LAPLACIAN, ks.KSUM_NEGDIST
    assert _st(10, 64, G) == ks.KSUM_OK
    assert _st(0, 64, G) == ks.KSUM_EINVAL
    assert _st(10, 0, G) == ks.KSUM_EINVAL
    assert ks.ksum_check_params(10, 4, 7, None) == ks.KSUM_EINVAL
    assert _st(10, 4, G, sigma=0.0) == ks.KSUM_EINVAL
    assert _st(10, 4, G, sigma=float("nan")) == ks.KSUM_EINVAL
    assert _st(10, 4, G, n_coeff=63) == ks.KSUM_EINVAL
    assert _st(10, 4, G, n_coeff=0) == ks.KSUM_EINVAL
    assert _st(10, 4, G, T=0.25) == ks.KSUM_EINVAL
    assert _st(10, 4, G, T=-0.1) == ks.KSUM_EINVAL
    assert _st(10, 4, G, coeff_eps=-1.0) == ks.KSUM_EINVAL
    assert _st(10, 4, G, method=9) == ks.KSUM_EINVAL
    assert _st(10, 4, G, method="sort") == ks.KSUM_EUNSUPPORTED
    assert _st(10, 4, N, method="nfft") == ks.KSUM_EUNSUPPORTED
    assert _st(10, 4, N, sigma=0.0) == ks.KSUM_OK               # sigma unused by the negative distance
    assert _st(10, 4, G, precision=1) == ks.KSUM_OK
    assert _st(10, 4, G, precision=5) == ks.KSUM_EINVAL
    assert _st(10, 4, G, slice_batch=-1) == ks.KSUM_EINVAL
    assert _st(10, 4, G, method="nfft", n_coeff=128, oversample=3) == ks.KSUM_EUNSUPPORTED   # grid not 2^k
    assert _st(10, 4, G, method="nfft", window_m=1) == ks.KSUM_EINVAL
    assert _st(10, 4, G, method="nfft", n_coeff=128, T=0.02) == ks.KSUM_OK
    assert _st(3072, 512, L) == ks.KSUM_OK
    assert _st(10, 4, G, check_finite=1) == ks.KSUM_OK
    assert _st(10, 4, N, check_finite=2) == ks.KSUM_EINVAL
    assert _st(10, 4, G, check_finite=-1) == ks.KSUM_EINVAL
    assert ks.ksum_last_error() != ""


def test_workspace_bytes_and_errors():
    b1 = ks.ksum_workspace_bytes(784, 256, ks.KSUM_NEGDIST, None, 1000, 1000)
    b2 = ks.ksum_workspace_bytes(784, 256, ks.KSUM_NEGDIST, None, 100000, 100000)
    assert 0 < b1 < b2
    # batching bounds the workspace
    b3 = ks.ksum_workspace_bytes(784, 256, ks.KSUM_NEGDIST, ks.make_params(ks.KSUM_NEGDIST, slice_batch=16),
                                 100000, 100000)
    assert b3 < b2 / 8
    with pytest.raises(ks.KsumError) as e:
        ks.ksum_workspace_bytes(784, 256, ks.KSUM_NEGDIST, None, 0, 10)
    assert e.value.status == ks.KSUM_EINVAL


def test_plan_create_without_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(ks.KsumError) as e:
        ks.ksum_plan_create(10, 4, ks.KSUM_NEGDIST)
    assert e.value.status == ks.KSUM_EDEVICE
    with pytest.raises(ks.KsumError) as e:
        ks.ksum_plan_create(0, 4, ks.KSUM_NEGDIST)
    assert e.value.status == ks.KSUM_EINVAL
