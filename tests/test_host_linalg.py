"""The coarse set-up's host-side inverse of a Hermitian positive definite
matrix (profile Cholesky factorisation within the envelope of the lower
triangle, column solves spread over threads), built with g++ from its
header and compared with numpy's dense inverse on block-banded, dense,
diagonal and irregular-envelope matrices; a matrix that is not positive
definite is rejected."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("hostla") / "hostla_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", os.path.join(HERE, "hostla_driver.cpp"), "-o", exe],
                   check=True)
    return exe


def _run(driver, G, tmp_path, threads):
    n = G.shape[0]
    src, dst = tmp_path / "G.bin", tmp_path / "Gi.bin"
    with open(src, "wb") as f:
        np.array([n], np.int32).tofile(f)
        np.ascontiguousarray(G, np.complex128).tofile(f)
    subprocess.run([driver, str(src), str(dst), str(threads)], check=True)
    raw = np.fromfile(dst, dtype=np.uint8)
    ok = int(raw[:4].view(np.int32)[0])
    if not ok:
        return None
    return raw[4:].view(np.complex128).reshape(n, n)


def _hpd_from_mask(mask, rng):
    """W^H W + small shift, with W's column couplings restricted to mask."""
    n = mask.shape[0]
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * mask
    G = A.conj().T @ A
    G = 0.5 * (G + G.conj().T) * (np.abs(G) > 0) + n * np.eye(n)
    return G


def _band_mask(n, w):
    i = np.arange(n)
    return (np.abs(i[:, None] - i[None, :]) <= w).astype(float)


@pytest.mark.parametrize("kind,threads", [("band", 1), ("band", 4), ("dense", 3), ("diag", 2), ("irregular", 5)])
def test_profile_inverse_matches_dense_inverse(driver, tmp_path, kind, threads):
    rng = np.random.default_rng(17)
    n = 150
    if kind == "band":
        G = _hpd_from_mask(_band_mask(n, 9), rng)
    elif kind == "dense":
        G = _hpd_from_mask(np.ones((n, n)), rng)
    elif kind == "diag":
        G = np.diag(rng.uniform(0.5, 2.0, n)).astype(np.complex128)
    else:
        # blocks of 4 columns coupled to a few earlier blocks at irregular
        # distances, as a quad-tree partition's neighbour lists give
        m = np.eye(n)
        for b in range(n // 4):
            for nb in rng.choice(max(b, 1), size=min(b, 3), replace=False) if b else []:
                m[4 * b:4 * b + 4, 4 * nb:4 * nb + 4] = 1
                m[4 * nb:4 * nb + 4, 4 * b:4 * b + 4] = 1
        A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * m
        G = A.conj().T @ A + n * np.eye(n)
    Gi = _run(driver, G, tmp_path, threads)
    assert Gi is not None
    ref = np.linalg.inv(G)
    assert np.linalg.norm(Gi - ref) / np.linalg.norm(ref) < 1e-12
    assert np.linalg.norm(G @ Gi - np.eye(n)) < 1e-10


def test_not_positive_definite_is_rejected(driver, tmp_path):
    rng = np.random.default_rng(3)
    G = _hpd_from_mask(_band_mask(40, 3), rng)
    G[20, 20] = -1.0
    assert _run(driver, G, tmp_path, 2) is None
