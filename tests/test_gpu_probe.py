"""ALU throughput probes on the GPU: plausible, positive rates."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_alu_rates_are_plausible():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10440_amd import probe
    r = probe.alu_rates(blocks=512, iters=1024)
    print("alu rates", {k: (f"{v:.3g}" if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    sys.stdout.flush()
    # 256 CUs x 2.4 GHz x 128 lanes bounds one FP32 instruction kind per cycle
    for k in ("fma", "fma_sgpr", "sin", "cos", "rcp"):
        assert 1e11 < r[k] < 256 * 2.4e9 * 128 * 1.05
    assert r["sin"] <= r["fma"] * 1.05
    assert 0.3 < r["mix_over_sum"] < 1.5
