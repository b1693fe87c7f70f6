"""The 2-bit pack codec on the GPU (gwfa_pack_dev) against a plain numpy
packing: A/a 0, C/c 1, G/g 2, T/t 3, 32 bases per 64-bit word with the first
base in the two most significant bits, zero-filled last word and a 2-word
zero tail; bit-exact at ragged sizes (every chunk slot of a wave, several
blocks, the full cfg2 read store size), from an unaligned start, and with a
base outside the alphabet reported."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

_CODE = np.zeros(256, np.uint64)
for i, c in enumerate("ACGT"):
    _CODE[ord(c)] = i
    _CODE[ord(c.lower())] = i


def say(msg):
    print(f"[gpu-pack] {msg}", flush=True)


def ref_pack(b: np.ndarray, words: int) -> np.ndarray:
    """The packed store by definition, 1 M bases at a time."""
    out = np.zeros(words, np.uint64)
    shifts = (62 - 2 * np.arange(32, dtype=np.uint64)).astype(np.uint64)
    step = 1 << 20
    for s in range(0, len(b), step):
        chunk = b[s:s + step]
        codes = _CODE[chunk]
        pad = (-len(codes)) % 32
        codes = np.concatenate([codes, np.zeros(pad, np.uint64)]).reshape(-1, 32)
        out[s // 32:s // 32 + len(codes)] = np.bitwise_or.reduce(codes << shifts, axis=1)
    return out


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def _pack(gw, ctx, host: np.ndarray, shift: int = 0):
    """Packs host[shift:] from a device buffer starting `shift` bytes in."""
    torch = ctx.torch
    n = len(host) - shift
    d = torch.from_numpy(host if len(host) else np.zeros(1, np.uint8)).to(ctx.tdev)
    words = gw.packed_words(n)
    out = torch.full((words,), -1, dtype=torch.int64, device=ctx.tdev)   # garbage the kernel must overwrite
    err = torch.zeros(1, dtype=torch.int32, device=ctx.tdev)
    rc = gw._lib.gwfa_pack_dev(ctx.h, ctypes.c_void_p(d.data_ptr() + shift), n, gw._tptr(out), gw._tptr(err),
                               ctypes.c_void_p(ctx.stream.cuda_stream))
    assert rc == 0
    torch.cuda.synchronize(ctx.tdev)
    return out.cpu().numpy().view(np.uint64), int(err.cpu().item())


def test_pack_ragged_sizes(G):
    gw, ctx = G
    rng = np.random.default_rng(71)
    sizes = [0, 1, 15, 16, 17, 31, 32, 33, 63, 64, 65, 1023, 1024, 1025, 4095, 4096, 4097, 16383, 16385,
             65536 + 13, 1_000_003]
    say(f"{len(sizes)} sizes, aligned and unaligned starts")
    for n in sizes:
        for shift in (0, 1, 7):
            host = np.frombuffer(b"ACGTacgt", np.uint8)[rng.integers(0, 8, size=n + shift)].copy()
            got, err = _pack(gw, ctx, host, shift)
            assert err == 0, (n, shift)
            assert np.array_equal(got, ref_pack(host[shift:], gw.packed_words(n))), (n, shift)


def test_pack_full_cfg2_store_size(G):
    """226.7 M bases, the size of the cfg2 read store, bit-exact."""
    gw, ctx = G
    from paper_2206_13574_amd import synth
    _, r = synth.cfg2()
    say(f"cfg2 read store: {len(r.seq)} bases")
    got, err = _pack(gw, ctx, np.ascontiguousarray(r.seq, np.uint8))
    assert err == 0
    assert np.array_equal(got, ref_pack(np.ascontiguousarray(r.seq, np.uint8), gw.packed_words(len(r.seq))))


def test_pack_reports_bases_outside_the_alphabet(G):
    gw, ctx = G
    rng = np.random.default_rng(72)
    say("bases outside ACGT")
    for n, pos, bad in ((1, 0, b"N"), (33, 32, b"n"), (5000, 4097, b"-"), (70000, 69999, b"\x00"),
                        (70000, 12345, b"U")):
        host = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=n)].copy()
        host[pos] = bad[0]
        _, err = _pack(gw, ctx, host)
        assert err == gw.ERR_ALPHABET, (n, pos, bad)
