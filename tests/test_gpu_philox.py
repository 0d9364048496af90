"""The library's random-stream checksum (hp_philox_xor) against the oracle's
independent Philox4x32-10: the sweeps' counter layout and key, both phases,
an odd block count (the single-block tail), t across 2^32."""
import numpy as np
import pytest

from oracle.philox import philox4x32
from tests.parity import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("phase", [0, 1])
def test_philox_xor_matches_oracle(hip, phase):
    import torch
    from paper_2311_02101_amd import hp
    seed, formula, t, chain = 0x1234_5678_9ABC_DEF0, 3, (1 << 32) + 17, 5
    blocks, n_out = 7, 33
    say(f"[philox xor] phase {phase}: {n_out} x {blocks} blocks")
    out = torch.zeros(n_out, dtype=torch.int32, device="cuda")
    hp.philox_xor(seed, formula, t, chain, phase, blocks, n_out, out)
    got = out.cpu().numpy().view(np.uint32)
    idx = np.arange(n_out * blocks, dtype=np.uint64)
    key = (seed & 0xFFFFFFFF, ((seed >> 32) ^ formula) & 0xFFFFFFFF)
    ctr = (np.uint64(t & 0xFFFFFFFF), np.uint64(chain), (np.uint64(phase) << np.uint64(31)) | idx,
           np.uint64(t >> 32))
    words = philox4x32(ctr, key).astype(np.uint32)                      # [n_out * blocks][4]
    want = np.bitwise_xor.reduce(words.reshape(n_out, blocks * 4), axis=1)
    assert np.array_equal(got, want)
