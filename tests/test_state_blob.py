"""Saved-state blobs are checked on the host before anything touches a
device: magic, version, declared and actual size, section counts and the
checksum (CPU only; the round trip through a context is a GPU test)."""
import struct

import numpy as np
import pytest

from paper_2504_12858_amd import binding as B

HEADER = struct.Struct("<IIQQd3d3ddqqqqq")
RECORD = {"grains": 56, "sites": 72, "particles": 24, "claims": 144}


def fnv1a64_words(payload: bytes) -> int:
    h = 0xcbf29ce484222325
    for (w,) in struct.iter_unpack("<Q", payload):
        h = ((h ^ w) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def pad8(n):
    return (n + 7) // 8 * 8


def make_blob(n_grains=2, n_sites=3, n_particles=5, n_claims=1, version=1, magic=0x54534547,
              seed=0):
    """A blob in the documented layout with arbitrary section contents."""
    g = np.random.default_rng(seed)
    sections = b""
    for name, n in (("grains", n_grains), ("sites", n_sites), ("particles", n_particles),
                    ("claims", n_claims)):
        raw = g.integers(0, 256, size=n * RECORD[name], dtype=np.uint8).tobytes()
        sections += raw + b"\0" * (pad8(len(raw)) - len(raw))
    total = HEADER.size + len(sections)
    hdr = HEADER.pack(magic, version, total, fnv1a64_words(sections), 5e-6,
                      0.0, 0.0, 0.0, 1e-3, 2e-3, 3e-3, 0.25, 17, n_grains, n_sites,
                      n_particles, n_claims)
    return bytearray(hdr + sections)


def check(blob):
    return B.state_check(np.frombuffer(bytes(blob), np.uint8))


def test_header_is_128_bytes():
    assert HEADER.size == 128


def test_valid_blob_is_accepted_and_read():
    blob = make_blob()
    h = check(blob)
    assert h["magic"] == B.STATE_MAGIC and h["version"] == B.STATE_VERSION
    assert h["bytes"] == len(blob)
    assert (h["n_grains"], h["n_sites"], h["n_particles"], h["n_claim_bricks"]) == (2, 3, 5, 1)
    assert h["t"] == 0.25 and h["step"] == 17 and h["hi"] == [1e-3, 2e-3, 3e-3]
    # An empty state is a valid blob too.
    assert check(make_blob(0, 0, 0, 0))["bytes"] == 128


def _rejected(blob):
    with pytest.raises(B.GrainEnvError) as e:
        check(blob)
    assert e.value.status == B.GE_EINVAL


def test_wrong_magic_or_version_is_rejected():
    _rejected(make_blob(magic=0x54534548))
    _rejected(make_blob(version=2))
    _rejected(make_blob(version=0))


def test_wrong_size_is_rejected():
    blob = make_blob()
    _rejected(blob[:-8])                 # truncated
    _rejected(blob + b"\0" * 8)          # trailing bytes
    _rejected(blob[:100])                # shorter than a header
    # Declared size that disagrees with the counts (the counts say more).
    _rejected(make_blob(n_particles=5)[:HEADER.size] + make_blob(n_particles=4)[HEADER.size:])


def test_counts_that_do_not_match_the_size_are_rejected():
    blob = make_blob()
    hdr = list(HEADER.unpack_from(blob))
    hdr[-2] = 6  # one particle more than the sections hold
    _rejected(HEADER.pack(*hdr) + bytes(blob[HEADER.size:]))
    hdr[-2] = -1
    _rejected(HEADER.pack(*hdr) + bytes(blob[HEADER.size:]))


def test_corrupted_payload_is_rejected():
    blob = make_blob()
    for at in (HEADER.size, HEADER.size + 57, len(blob) - 1):
        bad = bytearray(blob)
        bad[at] ^= 0x10
        _rejected(bad)
