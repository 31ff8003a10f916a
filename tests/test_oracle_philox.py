"""Pins for the oracle's Philox4x32-10: the generator's published known-answer vectors."""
import numpy as np

from oracle import philox

M = 0xFFFFFFFF


def test_known_answer_vectors():
    # counter, key -> output, from the known-answer tests distributed with the
    # generator's reference implementation (Random123)
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((M, M, M, M), (M, M), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = philox.philox4x32_10(*[np.array([v]) for v in ctr], *key)
        assert [int(g[0]) for g in got] == list(want)


def test_uniform53_is_exact_and_in_range():
    assert philox.u53(0, 0) == 0.0
    top = philox.u53(M, M)
    assert top == (2.0 ** 53 - 1) / 2.0 ** 53 and top < 1.0
    d = philox.perturbation_diagonal(100000, 20240704)
    assert d.min() >= 0.0 and d.max() < 1.0
    assert abs(d.mean() - 0.5) < 5e-3 and abs(d.var() - 1.0 / 12.0) < 2e-3


def test_start_block_is_standard_normal():
    om = philox.start_block(200000, 2, 7)
    assert om.flags.f_contiguous and om.shape == (200000, 2)
    for j in range(2):
        assert abs(om[:, j].mean()) < 1e-2 and abs(om[:, j].std() - 1.0) < 1e-2
    # the two columns come from different counter streams
    assert abs(np.corrcoef(om[:, 0], om[:, 1])[0, 1]) < 1e-2
