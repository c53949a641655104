"""fiuncho_scan_batch_static (no device allocation; the library's static
scratch as workspace) against fiuncho_scan_batch (caller workspace) through
the C ABI: two calls in a row, the second with smaller jobs, each with the
same bytes as the workspace entry point's results (and the oracle's)."""
import numpy as np
import pytest
import torch

from paper_2201_03331_amd import fiuncho, synth
from test_gpu_parity import check_hits_against_oracle, say

pytestmark = pytest.mark.gpu


def _static_vs_workspace(jobs):
    ref = fiuncho.DeviceBatch(jobs)
    ref.run()
    want = ref.results()
    got_b = fiuncho.DeviceBatch(jobs)
    for o in got_b.out:
        o.fill_(0xEE)
    got_b.run_static()
    got = got_b.results()
    for d, (s1, h1), (s2, h2) in zip(jobs, want, got):
        assert s1 == 0 and s2 == 0, (s1, s2)
        assert h1.tobytes() == h2.tobytes(), d.name
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, h2)
    torch.cuda.synchronize()


def test_static_scratch_two_calls_second_smaller():
    first = [synth.generate(300, 2000, seed=61, order=3, top_n=50, planted=[(3, 0.2)], name="s3"),
             synth.generate(150, 999, seed=62, order=2, top_n=20, case_fraction=0.4, name="s2")]
    second = [synth.order2_small()]
    shapes = [(d.n, d.m, d.order, d.top_n) for d in first]
    need = fiuncho.workspace_bytes(shapes)
    say(f"case: static scratch, first call {shapes} ({need} bytes of "
        f"{fiuncho.STATIC_SCRATCH_BYTES}), then {[(d.n, d.m, d.order, d.top_n) for d in second]}")
    assert fiuncho.workspace_bytes([(d.n, d.m, d.order, d.top_n) for d in second]) < need
    assert need <= fiuncho.STATIC_SCRATCH_BYTES
    _static_vs_workspace(first)
    _static_vs_workspace(second)
