"""Pins of the oracle's ChaCha20 keystream family against OpenSSL's ChaCha20
(a library routine independent of the oracle), run through the openssl
command-line tool: encrypting zero bytes returns the keystream.  OpenSSL's
16-byte IV for ChaCha20 is the 32-bit block counter (little-endian) followed
by the 96-bit nonce, the IETF layout the oracle uses."""
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl tool not available")


def _openssl_stream(key: bytes, counter: int, nonce: bytes, nbytes: int) -> np.ndarray:
    iv = counter.to_bytes(4, "little") + nonce
    r = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                       input=bytes(nbytes), capture_output=True, check=True)
    assert len(r.stdout) == nbytes
    return np.frombuffer(r.stdout, dtype=np.uint8)


def _words(b: bytes) -> np.ndarray:
    return np.frombuffer(b, dtype="<u4").astype(np.uint32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chacha20_block_matches_openssl(seed):
    """The block function for random keys, nonces and counters (including a
    counter next to 2^32, where OpenSSL's counter wraps past this block only)."""
    rng = np.random.default_rng(seed)
    key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
    nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
    counter = [0, 7, 0xFFFFFFFE][seed]
    want = _openssl_stream(key, counter, nonce, 64)
    got = O.chacha20_block(_words(key), counter, _words(nonce))
    assert np.array_equal(got, want)


def test_chacha20_zero_key_block():
    """All-zero key, nonce and counter: the block OpenSSL gives, and not the
    Philox stream (the family switch takes effect)."""
    want = _openssl_stream(bytes(32), 0, bytes(12), 64)
    assert np.array_equal(O.chacha20_block(np.zeros(8, np.uint32), 0, np.zeros(3, np.uint32)), want)


@pytest.mark.parametrize("key,domain,first,count", [
    (0x0123456789ABCDEF, 1, 0, 1000),
    (0xFEDCBA9876543210, 2, 64 * 5 + 17, 300),
    (42, 1, (1 << 36) - 200, 200),          # the last bytes of the longest stream the oracle draws
])
def test_keystream_family_is_the_ietf_chacha20_stream(key, domain, first, count):
    """Byte idx of stream (key, nonce 0, domain) is byte idx of the RFC 8439
    keystream with key = K as 8 little-endian bytes then 24 zero bytes, nonce =
    (domain, 0, 0) as little-endian words, counter from 0."""
    kb = key.to_bytes(8, "little") + bytes(24)
    nonce = domain.to_bytes(4, "little") + bytes(8)
    c0 = first // 64
    span = (first + count + 63) // 64 - c0
    ref = _openssl_stream(kb, c0, nonce, 64 * span)[first - 64 * c0:first - 64 * c0 + count]
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        got = O.keystream(key, domain, first, count)
    assert np.array_equal(got, ref)
    assert not np.array_equal(O.keystream(key, domain, first, count), ref)   # back to Philox


@pytest.mark.parametrize("nonce", [1, 0x89ABCDEF, 0x0123456789ABCDEF, (1 << 64) - 1])
def test_keystream_nonce_fills_ietf_nonce_words_1_and_2(nonce):
    """The per-image nonce is the second and third word of the RFC 8439 nonce:
    stream (key, nonce, domain) is OpenSSL's keystream with nonce bytes
    domain, nonce low word, nonce high word (little-endian)."""
    key, domain = 0x1122334455667788, 2
    kb = key.to_bytes(8, "little") + bytes(24)
    nb = domain.to_bytes(4, "little") + (nonce & 0xFFFFFFFF).to_bytes(4, "little") + (nonce >> 32).to_bytes(4, "little")
    ref = _openssl_stream(kb, 3, nb, 192)[7:7 + 150]
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        got = O.keystream(key, domain, 3 * 64 + 7, 150, nonce)
        zero = O.keystream(key, domain, 3 * 64 + 7, 150, 0)
    assert np.array_equal(got, ref)
    assert not np.array_equal(got, zero)


def test_chacha_round_trip_in_the_oracle():
    """EMR encrypt / embed / extract / recover under ChaCha20: the payload
    comes back, the image comes back above the LSB plane, and the encrypted
    image differs from the Philox one."""
    rng = np.random.default_rng(3)
    y, x = np.indices((64, 96))
    I = np.clip(120 + 50 * np.sin(x / 9.0) + rng.normal(0, 3, (64, 96)), 0, 255).astype(np.uint8)
    Ie_p, _ = O.emr_encrypt(I, 11)
    with O.keystream_family(O.KEYSTREAM_CHACHA20):
        Ie, meta = O.emr_encrypt(I, 11)
        nbits = min(int(meta.capacity_bits), 5000)
        msg = rng.integers(0, 256, (nbits + 7) // 8).astype(np.uint8)
        Iw = O.emr_embed(Ie, meta.b, msg, nbits, 22)
        got = O.emr_extract(Iw, meta.b, nbits, 22)
        rec = O.emr_recover(Iw, meta.b, 11)
    assert not np.array_equal(Ie, Ie_p)
    full, rest = nbits // 8, nbits % 8
    assert np.array_equal(got[:full], msg[:full])
    if rest:
        assert (got[full] >> (8 - rest)) == (msg[full] >> (8 - rest))
    assert np.array_equal(rec >> 1, I >> 1)
