"""GPU tests of the FGP autotuner and its JSON tuning files.

The FGP variants give bitwise identical results (same per-pixel arithmetic,
different tiling), so tuning only changes speed; these tests check which
variant each size picks up (exact entry, size class, default), the file
round trip and the error paths (the table is unchanged after a bad file).
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2411_00688_amd as T
from paper_2411_00688_amd._lib import TVS_F32, TVS_F64

pytestmark = pytest.mark.gpu


def variant_index(tile_w, tile_h, steps):
    for i in range(T.tvs_fgp_variant_count()):
        if T.tvs_fgp_variant(i) == (tile_w, tile_h, steps):
            return i
    raise AssertionError("variant not compiled")


@pytest.fixture
def tctx():
    c = T.tvs_ctx_create(0)
    yield c
    T.tvs_ctx_destroy(c)


def test_autotune_exact_class_and_default(tctx):
    default = variant_index(32, 32, 4)
    best, ms = T.tvs_fgp_autotune(tctx, TVS_F32, 48, 40, 8, 2)
    assert 0 <= best < T.tvs_fgp_variant_count() and ms[best] == min(m for m in ms if m >= 0)
    idx, m = T.tvs_fgp_query(tctx, TVS_F32, 48, 40)
    assert idx == best and m == pytest.approx(ms[best])
    # same size class (64, 64): the class entry
    assert T.tvs_fgp_query(tctx, TVS_F32, 60, 33)[0] == best
    # another class, another dtype: the default
    assert T.tvs_fgp_query(tctx, TVS_F32, 100, 100) == (default, -1.0)
    assert T.tvs_fgp_query(tctx, TVS_F64, 48, 40) == (default, -1.0)
    # a hand-set exact entry overrides the class entry for that size only
    other = (best + 1) % T.tvs_fgp_variant_count()
    if other == variant_index(64, 32, 8):
        other = default
    T.tvs_fgp_set_variant(tctx, TVS_F32, 60, 33, other)
    assert T.tvs_fgp_query(tctx, TVS_F32, 60, 33) == (other, -1.0)
    assert T.tvs_fgp_query(tctx, TVS_F32, 64, 64)[0] == best


def test_tuning_file_round_trip_and_errors(tctx, tmp_path):
    T.tvs_fgp_autotune(tctx, TVS_F32, 40, 40, 4, 1)
    T.tvs_fgp_set_variant(tctx, TVS_F64, 17, 9, variant_index(16, 16, 4))
    T.tvs_fgp_set_variant_batched(tctx, TVS_F32, 12, variant_index(64, 16, 1))
    path = os.path.join(tmp_path, "tune.json")
    T.tvs_tune_save(tctx, path)
    doc = json.load(open(path))
    assert doc["format"] == "tvskip-fgp-tune/1" and doc["arch"].startswith("gfx")
    kinds = sorted(e["kind"] for e in doc["entries"])
    assert kinds == ["batch", "class", "image", "image"]
    before = (T.tvs_fgp_query(tctx, TVS_F32, 40, 40), T.tvs_fgp_query(tctx, TVS_F64, 17, 9),
              T.tvs_fgp_query_batched(tctx, TVS_F32, 12), T.tvs_fgp_query(tctx, TVS_F32, 50, 60))
    T.tvs_tune_clear(tctx)
    assert T.tvs_fgp_query(tctx, TVS_F64, 17, 9)[1] == -1.0
    T.tvs_tune_load(tctx, path)
    after = (T.tvs_fgp_query(tctx, TVS_F32, 40, 40), T.tvs_fgp_query(tctx, TVS_F64, 17, 9),
             T.tvs_fgp_query_batched(tctx, TVS_F32, 12), T.tvs_fgp_query(tctx, TVS_F32, 50, 60))
    assert after == before
    # error paths leave the table as it is
    bad = os.path.join(tmp_path, "bad.json")
    for text, status in [("{\"format\": \"tvskip-fgp-tune/1\", \"arch\": ", 1),
                         (json.dumps({**doc, "arch": "gfx000"}), 6),
                         (json.dumps({**doc, "entries": [{**doc["entries"][0], "steps": 3}]}), 6),
                         (json.dumps({**doc, "format": "other"}), 1),
                         (json.dumps({**doc, "entries": [{"kind": "image", "dtype": "f32"}]}), 1)]:
        open(bad, "w").write(text)
        with pytest.raises(T.TvsError) as ei:
            T.tvs_tune_load(tctx, bad)
        assert ei.value.status == status, text
        assert (T.tvs_fgp_query(tctx, TVS_F32, 40, 40), T.tvs_fgp_query(tctx, TVS_F64, 17, 9),
                T.tvs_fgp_query_batched(tctx, TVS_F32, 12),
                T.tvs_fgp_query(tctx, TVS_F32, 50, 60)) == before


def test_batched_autotune_changes_speed_not_results(tctx):
    sizes = [(40, 33), (64, 64), (17, 80), (96, 50)]
    slices, off = [], 0
    rng = np.random.default_rng(1)
    for s, (H, W) in enumerate(sizes):
        slices.append(dict(H=H, W=W, offset=off, alpha=0.1, p=0.5, seed=s, stream_id=s))
        off += H * W
    best, ms = T.tvs_fgp_autotune_batched(tctx, TVS_F32, slices, 8, 2)
    assert T.tvs_fgp_query_batched(tctx, TVS_F32, len(slices)) == (best, pytest.approx(ms[best]))
    b = torch.tensor(rng.random(off), dtype=torch.float32, device="cuda")
    outs = []
    for fv in (-1, variant_index(32, 32, 1)):
        x, h = torch.zeros(off, device="cuda"), torch.zeros(off, device="cuda")
        q = torch.zeros(2 * off, device="cuda")
        T.tvs_proxskip_batched(tctx, slices, b, x, h, q, 1.0, 20, 10, fgp_variant=fv)
        outs.append(x)
    assert torch.equal(outs[0], outs[1])
