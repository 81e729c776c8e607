"""Oracle pins: counter-based random numbers and lattice rotations.

Philox4x64-10 is checked against numpy's independent implementation; the
rotation against the defining properties of a uniform rotation.
"""
import numpy as np
import pytest

import oracle
from paper_1909_01589_amd.inputs import hydrogenic


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle.Oracle(hydrogenic(1.0), a=0.1, a_prime=0.1, r_c=1.0, seed=7)


def _numpy_block(key, ctr):
    """numpy's Philox increments its 256-bit counter before each block, so
    block c is produced by a generator started at c - 1."""
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((7, 0), (3, 11, 0, 1)),
    ((2**64 - 1, 0), (2**64 - 1, 5, 2**40, 3)),
    ((123456789, 0), (4095, 1999, 37, 0)),
    ((0xDEADBEEF, 0), (2**63, 2**63 + 1, 17, 2)),
])
def test_philox_matches_numpy(orc, key, ctr):
    assert np.array_equal(orc.philox(ctr, key), _numpy_block(key, ctr))


def test_u01_open_interval_and_resolution(orc):
    lib = orc.lib
    assert lib.orc_u01(0) == 0.5 * 2.0 ** -53
    assert lib.orc_u01(2**64 - 1) == 1.0 - 0.5 * 2.0 ** -53
    assert 0.0 < lib.orc_u01(2**63) < 1.0
    assert lib.orc_u01(2**63) == 0.5 + 0.5 * 2.0 ** -53


def test_draws_are_uniform(orc):
    u = np.array([orc.draw(s, 3, 9, 0) for s in range(4000)]).ravel()
    assert np.all((u > 0) & (u < 1))
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    expected = u.size / 20
    chi2 = np.sum((hist - expected) ** 2 / expected)
    assert chi2 < 45.0  # 19 dof, p ~ 1e-3


def test_rotation_is_proper_orthogonal(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        R = orc.rotation(rng.uniform(size=3))
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14


def test_rotation_is_uniform(orc):
    """A uniform rotation maps a fixed axis to a uniform direction: mean 0,
    second moment I/3, and the trace of R has the Haar mean 0."""
    Rs = np.array([orc.move_rotation(s, 0, 0) for s in range(20000)])
    e1 = Rs[:, :, 0]
    assert np.all(np.abs(e1.mean(axis=0)) < 0.03)
    assert np.allclose(e1.T @ e1 / len(e1), np.eye(3) / 3, atol=0.02)
    assert abs(np.trace(Rs, axis1=1, axis2=2).mean()) < 0.03


def _u01(x):
    return ((int(x) >> 11) + 0.5) * 2.0 ** -53


def test_stream_layout_against_numpy(orc):
    """Counter layout (slot, generation, iteration, purpose) with key (seed, 0):
    purpose 0 gives (u1, u2) of a move, 1 the rotation, 3 the resampling
    offset xi at slot 2^64 - 1."""
    seed = orc.prm.seed
    for slot, gen, it in ((0, 0, 0), (5, 17, 3), (4095, 1999, 40)):
        for purpose in (0, 1):
            blk = _numpy_block((seed, 0), (slot, gen, it, purpose))
            assert np.array_equal(orc.draw(slot, gen, it, purpose), [_u01(x) for x in blk])
    for gen in (0, 1, 977):
        blk = _numpy_block((seed, 0), (2**64 - 1, gen, 0, 3))
        assert orc.xi(gen) == _u01(blk[0])
