"""The autotuner's sweep on a small batch: it records an entry with every
launch choice, `apply` restores that entry on a fresh code object, and the
tuned decode equals the decode with the library defaults (every launch choice
gives identical results)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1008_4370_amd import autotune, synth  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402

pytestmark = pytest.mark.gpu


def test_tune_records_an_entry_that_apply_restores(tmp_path):
    b = synth.make_batch("gf4_n96", frames=256)
    print("[case] autotune gf4_n96 256 frames", flush=True)
    llr = torch.from_numpy(b.llr).cuda()
    path = str(tmp_path / "tuned.json")
    code = D.Code.from_synth(b.code)
    ent = autotune.tune(code, llr, "fp32", 50, reps=1, grid_blocks=(2048, 8192), chunks=(4, 8),
                        tail_frames=(32, 1 << 20), tail_chunks=(0, 16), path=path)
    code.close()
    for k in ("lane_entries", "grid_blocks", "chunk", "first_chunk", "tail_entries", "tail_frames", "tail_chunk",
              "batch_retire", "ms"):
        assert k in ent, k
    tuned = D.Code.from_synth(b.code)
    assert autotune.apply(tuned, "fp32", 256, path=path) is not None
    t = tuned.get_tuning()
    for k in ("lane_entries", "grid_blocks", "chunk", "first_chunk", "tail_entries", "tail_frames", "tail_chunk",
              "batch_retire"):
        assert t[k] == ent[k], k
    plain = D.Code.from_synth(b.code)
    r1 = {k: v.cpu().numpy() for k, v in D.decode(tuned, llr, 50, prec="fp32").items()}
    r0 = {k: v.cpu().numpy() for k, v in D.decode(plain, llr, 50, prec="fp32").items()}
    for k in r0:
        assert np.array_equal(r1[k], r0[k]), k
    tuned.close()
    plain.close()
