"""Known-answer vectors of Philox4x32-10 (published with the Random123
library of the SC'11 paper) for the pure-Python reference generator."""
from philox_ref import philox4x32_10


def test_kat_zero():
    assert philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)


def test_kat_ones():
    f = 0xFFFFFFFF
    assert philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)


def test_kat_pi():
    ctr = (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344)
    key = (0xA4093822, 0x299F31D0)
    assert philox4x32_10(ctr, key) == (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)
