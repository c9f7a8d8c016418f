"""Pin the oracle's ChaCha20 block function and stream layout to OpenSSL.

The keystream convention (ChaCha20 as in RFC 8439, 32-bit counter, 96-bit
nonce) is the library's own seed expansion; the paper only asks for uniform
random sampling (Section 3.1).  The reference values come from the host's
``openssl enc -chacha20`` command-line tool, a library routine independent of
the oracle.
"""
import shutil
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI missing")


def openssl_keystream(key: bytes, counter: int, nonce: bytes, nbytes: int) -> bytes:
    iv = counter.to_bytes(4, "little") + nonce
    out = subprocess.run(
        ["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
        input=bytes(nbytes), stdout=subprocess.PIPE, stderr=subprocess.PIPE, check=True)
    return out.stdout


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_block_matches_openssl(seed):
    rng = np.random.default_rng(1000 + seed)
    key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
    nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
    counter = int(rng.integers(0, 2**32 - 8))
    ref = openssl_keystream(key, counter, nonce, 64 * 4)
    for blk in range(4):
        assert oracle.chacha20_block(key, counter + blk, nonce) == ref[64 * blk:64 * blk + 64]


@pytest.mark.parametrize("p,stream,index", [(761, 0, 0), (761, 3, 12345), (1277, 64, 2**40 + 7)])
def test_stream_layout_matches_openssl(p, stream, index):
    """Word i of stream s of key `index` is the LE u32 at keystream offset 4i
    under nonce = index (u64 LE) || p (u16 LE) || s (u16 LE), counter from 0."""
    seed = bytes(range(32))
    nonce = index.to_bytes(8, "little") + p.to_bytes(2, "little") + stream.to_bytes(2, "little")
    ks = openssl_keystream(seed, 0, nonce, 4 * p)
    ref = np.frombuffer(ks, dtype="<u4")
    got = oracle.stream_words(seed, index, p, stream, p)
    assert np.array_equal(got, ref)
