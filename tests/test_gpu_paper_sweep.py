"""GPU parity on the paper's dataset families (Sec. III-B): uniform over k
values, rounded Gaussians as signed keys, Zipf(1.5), the edge patterns,
full-range signed keys and the stand-ins for the three real datasets, each
through AUTO (with and without payload) and the forced radix and general
paths, against the oracle.  Same bar as the other parity tests."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_20677_amd as ahs  # noqa: E402
from test_gpu_parity import run_pair  # noqa: E402


@pytest.mark.parametrize("case", gen.PAPER_CASES)
def test_paper_family_parity(case):
    n = (1 << 20) + 7 if case in gen.PAPER_REAL else (1 << 18) + 3
    keys = gen.paper_sweep(case, n=n)
    run_pair(keys, np.arange(n, dtype=np.uint32))
    run_pair(keys)
    run_pair(keys, None, ahs.RADIX)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)
