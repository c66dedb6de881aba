"""The no-allocation entry point through the C ABI against corr_process on
the same inputs: two calls in a row on one GPU (the second smaller, so it
runs over what the first left in the shared scratch array), each compared
with a fresh correlator's corr_read_cps_raw.  fp32 / fp16 within their
tolerance (the chunking and splits differ), int8 / int16 identical sums and
identical scales."""
import numpy as np
import pytest
import torch

import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import TOL, coef_error, raw_to_complex

pytestmark = pytest.mark.gpu

# (N, K, S): the first call runs several chunks with a ragged last one; the
# second is smaller in every dimension
CALLS = [(44, 256, 20000), (12, 128, 300)]


def _noalloc(N, K, S, prec, packed):
    code = corr.PRECISIONS[prec]
    nb = N * (N + 1) // 2
    cps = torch.full((nb * K * 2,), float("nan"), dtype=torch.float64, device="cuda")
    scales = torch.full((N * K,), float("nan"), dtype=torch.float32, device="cuda") if code >= corr.CORR_INT8 else None
    stream = torch.cuda.current_stream()
    corr.corr_process_noalloc(N, K, S, code, packed.data_ptr(), cps.data_ptr(),
                              None if scales is None else scales.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    raw = cps.cpu().numpy().reshape(nb, K, 2)
    return raw, (None if scales is None else scales.cpu().numpy().reshape(N, K))


def _reference(N, K, S, prec, packed):
    c = corr.Correlator(N, K, S, precision=prec)
    c.process(packed)
    sc = c.read_scales() if prec in ("int8", "int16") else None
    raw = c.read_cps_raw()
    c.close()
    return raw, sc


@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_noalloc_matches_corr_process_twice(prec):
    for i, (N, K, S) in enumerate(CALLS):
        print(f"\n[no-alloc] {prec} call {i}: N={N} K={K} S={S}", flush=True)
        recipe = synth.recipe_tone(N=N, two_k=2 * K, seed=40 + i, tone_bin=K // 3, tone_amp=0.5)
        packed = synth.packed(recipe, 0, S, device="cuda").contiguous()
        got, sc_got = _noalloc(N, K, S, prec, packed)
        ref, sc_ref = _reference(N, K, S, prec, packed)
        assert np.all(np.isfinite(got))
        if prec in ("fp32", "fp16"):
            err = coef_error(raw_to_complex(got), raw_to_complex(ref), N)
            print(f"  coefficient error against corr_process: {err:.3g}", flush=True)
            assert err <= TOL[corr.PRECISIONS[prec]]
        else:
            np.testing.assert_array_equal(sc_got, sc_ref)
            np.testing.assert_array_equal(got, ref)


def test_noalloc_rejects_what_does_not_fit():
    """N = 256 at K = 512: the float64 integration buffer alone (269 MB)
    exceeds the array; refused before anything is enqueued."""
    x = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(corr.CorrError) as e:
        corr.corr_process_noalloc(256, 512, 64, corr.CORR_FP32, x.data_ptr(), out.data_ptr(), None, 0)
    assert e.value.code == corr.CORR_EINVAL
    assert "bytes of scratch" in str(e.value)
