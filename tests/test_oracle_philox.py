"""Pins of oracle.philox: the Random123 known-answer vectors of Philox4x32-10
(kat_vectors: counter, key -> output) and the N(0,1) moments of the fields."""
import numpy as np

from oracle.philox import fields, philox4x32_10


def test_known_answer_vectors():
    # Random123 kat_vectors, philox4x32_10 (ctr[4], key[2] -> out[4])
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, out in cases:
        got = philox4x32_10(*ctr, *key)
        assert tuple(int(g) for g in got) == out


def test_fields_are_standard_normal():
    E, A = fields((3, 20, 30, 40), 12345)
    for z in (E.real, E.imag, A.real, A.imag):
        assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02
    E2, _ = fields((3, 20, 30, 40), 12346)
    assert not np.allclose(E, E2)
