"""ahs_sort_static (the entry point that allocates nothing: its scratch is
the library's fixed per-device array) against ahs_sort with a caller
workspace, bit for bit, on two calls in a row -- the second with a smaller
input, so stale scratch contents from the first call must not matter --
for AUTO and each forced strategy, keys only and with payload; plus the
size limit, which must be refused before any launch."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_20677_amd as ahs  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(kind, n, seed):
    if kind == "u32":
        return gen.u32(seed, 0, n)
    if kind == "u32small":
        return gen.u32(seed, 0, n, mask=1023)
    if kind == "u64zipf":
        return gen.zipf_keys(seed, n, 4096, 1.0, 64)
    if kind == "f32":
        return gen.normal(seed, 1, n, 1000.0).astype(np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("payload", [False, True])
@pytest.mark.parametrize("strategy", ["auto", "counting", "radix", "quick"])
@pytest.mark.parametrize("kind", ["u32", "u32small", "u64zipf", "f32"])
def test_static_matches_workspace_call(kind, strategy, payload):
    if strategy == "counting" and kind != "u32small":
        pytest.skip("counting sort needs a span below its cap")
    for call, n in enumerate((1_000_003, 77_777)):  # second call smaller than the first
        say(f"no-alloc {kind} {strategy} payload={payload} call {call} n={n}")
        keys = torch.from_numpy(_inputs(kind, n, 31 + call)).to(DEV)
        vals = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32) if payload else None
        out_s = torch.empty_like(keys)
        vout_s = torch.empty_like(vals) if payload else None
        torch.cuda.synchronize()
        ch_s, f_s = ahs.ahs_sort_static(keys, out_s, vals, vout_s, strategy=strategy, want_features=True)
        out_w, vout_w, ch_w, f_w = ahs.ahs_sort(keys, vals, strategy=strategy, want_features=True)
        torch.cuda.synchronize()
        assert ch_s == ch_w
        assert torch.equal(out_s.view(torch.uint8), out_w.view(torch.uint8)), "keys differ"
        if payload:
            assert torch.equal(vout_s.view(torch.int32), vout_w.view(torch.int32)), "payload differs"
        assert (f_s.n, f_s.min_key, f_s.max_key, f_s.span, f_s.nbins) == (f_w.n, f_w.min_key, f_w.max_key, f_w.span,
                                                                         f_w.nbins)
        assert f_s.entropy_bits == f_w.entropy_bits


def test_static_rejects_sizes_beyond_its_scratch():
    n = 1 << 23  # needs more than the 64 MiB scratch under AUTO
    assert ahs.ahs_workspace_bytes(n, ahs.U32, False, ahs.AUTO) > ahs.STATIC_SCRATCH_BYTES
    keys = torch.zeros(n, dtype=torch.int32, device=DEV).view(torch.uint32)
    out = torch.full_like(keys.view(torch.int32), 7).view(torch.uint32)
    torch.cuda.synchronize()
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_sort_static(keys, out)
    assert e.value.status == ahs.E_WORKSPACE
    torch.cuda.synchronize()
    assert bool((out.view(torch.int32) == 7).all().item()), "output written despite the refusal"
