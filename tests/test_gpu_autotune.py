"""The autotuner picks among choices that leave the results unchanged: a
batch run with the tuned configuration has the same contact sets as with the
defaults, and states within the FP32 tolerance."""
import numpy as np
import pytest

from paper_2211_01185_amd import autotune, cfddem, synth
from tests.parity_util import TOL, assert_close, gpu_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tuned_configuration_gives_the_same_results(tmp_path, monkeypatch):
    monkeypatch.setenv("CFDDEM_TUNE_CACHE", str(tmp_path / "tune.json"))
    wls = [synth.column_bed(synth.rng_for(4, 900 + j), n, d, 0.8, 1.0, precision="fp32")
           for j, (n, d) in enumerate([(4000, 1.5e-3), (2500, 2.2e-3)])]
    cfg, report = autotune.tune(wls, "fp32", steps=20)
    for k, v in cfg.items():
        assert v in autotune.CANDIDATES[k]
    assert report["trials"] >= 2 and not report["cached"]
    cfg2, report2 = autotune.tune(wls, "fp32", steps=20)
    assert cfg2 == cfg and report2["cached"]

    def run(c):
        fields = [(torch.as_tensor(w.U, device="cuda").contiguous(), torch.as_tensor(w.P, device="cuda").contiguous())
                  for w in wls]
        beds = [cfddem.bed_from_workload(w, precision="fp32", **autotune.bed_kwargs(w, c)) for w in wls]
        batch = cfddem.Batch(beds, fields)
        batch.run(5, 10, couple=True)
        out = [(b.read_contacts(), gpu_state(b)) for b in beds]
        batch.close()
        return out

    for (ca, sa), (cb, sb) in zip(run(cfg), run(autotune.DEFAULT)):
        assert np.array_equal(ca[0], cb[0]) and np.array_equal(ca[1], cb[1])
        for k in sa:
            assert_close(k, sa[k], sb[k], 10 * TOL["fp32"])
