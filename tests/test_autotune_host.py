"""Host-side logic of the autotuner: the cached table is keyed by the shape
of the problem and re-applied through hbf_tune without timing anything."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1901_11371_amd import autotune  # noqa: E402


class FakeCtx:
    def __init__(self, n=4096, dtype="c64", prec="block"):
        self.n, self.dtype, self.prec = n, dtype, prec
        self.calls = []

    def tune(self, k, v):
        self.calls.append((k, v))


def test_apply_uses_the_entry_of_the_same_shape(tmp_path):
    path = tmp_path / "table.json"
    ctx = FakeCtx()
    other = FakeCtx(n=8192)
    table = {
        autotune._key(ctx, 64): {"params": {"prog_levels": 6, "pipe_max_r": 0}, "kernel": "wave"},
        autotune._key(other, 64): {"params": {"prog_levels": 4}, "kernel": "pipe"},
    }
    path.write_text(json.dumps(table))
    entry = autotune.apply(ctx, 64, path=str(path))
    assert entry["kernel"] == "wave"
    assert ctx.calls == [("prog_levels", 6), ("pipe_max_r", 0)]
    # another RHS count is another shape: nothing applied
    ctx2 = FakeCtx()
    assert autotune.apply(ctx2, 1, path=str(path)) is None and ctx2.calls == []


def test_missing_or_broken_table_applies_nothing(tmp_path):
    ctx = FakeCtx()
    assert autotune.apply(ctx, 1, path=str(tmp_path / "missing.json")) is None
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.apply(ctx, 1, path=str(bad)) is None
    assert ctx.calls == []


def test_every_kernel_candidate_sets_the_same_keys():
    keys = None
    for name, fn in autotune.KERNELS.items():
        for R in (1, 64):
            s = fn(R)
            assert all(isinstance(v, int) for v in s.values()), name
            keys = keys or set(s)
            assert set(s) == keys, name
