"""The streaming-read ceiling kernel the benchmark compares the products with: it must read
every byte once (its per-workgroup folded words XOR to the XOR of all input words)."""
import numpy as np
import pytest
import torch

from paper_1108_0900_amd import sr
from tests.gpu_util import DEV

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_words", [4, 4 * 1000 + 4, 4 * (1 << 20) + 12])
def test_stream_read_visits_every_word_once(n_words):
    gen = torch.Generator().manual_seed(n_words)
    host = torch.randint(-2 ** 31, 2 ** 31 - 1, (n_words,), dtype=torch.int64, generator=gen).to(torch.int32)
    t = host.to(DEV)
    want = np.bitwise_xor.reduce(host.numpy().view(np.uint32))
    for bpc in (1, 2, 4):
        for unroll in (2, 4, 8):
            sink = sr.stream_read(t, bpc, unroll)
            got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
            assert got == want, (bpc, unroll)
