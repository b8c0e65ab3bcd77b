"""planb_lookup_learned_noalloc (the learned lookup whose fallback queue is a
fixed device array of the library) against planb_lookup_learned (queue from
the stream-ordered pool) through the C ABI: two calls in a row, the second
smaller, with the trained error bounds and with bounds forced to zero (many
window checks fail), so that the shared queue is used and keeps the previous
call's contents; for both learned kernels (64- and 128-bit key slots).
Next hops are integers: compared bit for bit, and with the LPM oracle."""
import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, host_u16, oracle_trie, say, to_dev

pytestmark = pytest.mark.gpu

LIMIT = 1 << 22  # lookups per call of the no-alloc entry point


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


@pytest.fixture(scope="module", params=[0, 128], ids=["keys64", "keys128"])
def trained(P, request):
    """64-bit key slots run the leaf-tops kernel, 128-bit ones the leaf-key window search."""
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8, key_bits=request.param)
    P.planb_train(h, seed=5)
    return fib, h


def _both(P, h, addrs):
    import torch
    n = len(addrs)
    d = to_dev(addrs)
    outs, fbs = [], []
    for fn in (P.planb_lookup_learned, P.planb_lookup_learned_noalloc):
        out = torch.full((n,), -1, dtype=torch.int16, device="cuda")
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        fn(h, d, n, out, fb)
        torch.cuda.synchronize()
        outs.append(host_u16(out, n))
        fbs.append(int(fb.item()))
    return outs, fbs


@pytest.mark.parametrize("forced", [False, True])
def test_noalloc_matches_learned_two_calls(P, trained, forced):
    fib, h = trained
    want_of = oracle_trie("tiny", 11)
    saved = P.planb_model_get_eps(h, 4096)
    try:
        if forced:  # error bounds of zero: many window checks fail, so the queue fills
            P.planb_model_set_eps(h, np.zeros(len(saved), np.uint32))
        for k, n in enumerate((LIMIT, 3001)):  # the second call is smaller
            addrs = S.tiny_traffic(fib, n, seed=700 + 10 * k + int(forced))
            say(f"no-alloc learned lookup: call {k}, n={n}, forced fallbacks={forced}")
            (ref, got), (fb_ref, fb_got) = _both(P, h, addrs)
            assert np.array_equal(got, ref)
            assert np.array_equal(got, want_of.lookup(addrs))
            assert fb_got == fb_ref
            if forced:
                assert fb_got > n // 100
    finally:
        P.planb_model_set_eps(h, saved)


def test_noalloc_rejects_more_than_its_queue(P, trained):
    import torch
    fib, h = trained
    d = torch.zeros((LIMIT + 1, 2), dtype=torch.int64, device="cuda")
    out = torch.empty(LIMIT + 1, dtype=torch.int16, device="cuda")
    with pytest.raises(P.PlanbError) as e:
        P.planb_lookup_learned_noalloc(h, d, LIMIT + 1, out)
    assert e.value.code == P.PLANB_ERANGE
    assert "at most" in str(e.value)
