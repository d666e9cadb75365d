"""Philox4x32-10 against the known-answer vectors published with the
generator (Salmon et al., SC'11, Random123 distribution)."""
import numpy as np

from oracle.philox import philox4x32_10, philox4x32_10_np

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_known_answers():
    for ctr, key, out in KAT:
        assert philox4x32_10(ctr, key) == out
        got = philox4x32_10_np(np.array([ctr], dtype=np.uint64), np.array([key], dtype=np.uint64))
        assert tuple(int(v) for v in got[0]) == out
