"""The stored tile geometry is keyed by (n, m) bucket: every bucket holds
options tuned on an MI355X, and any input (sizes never tuned included) gets
the options of the bucket holding it or of the nearest one."""

import json

from paper_2304_01660_amd import tuning

KEYS = {"dist_bits", "guard", "near_cols", "chunk_cols", "rows_near", "rows_far",
        "rows_refine", "far_grid", "band_pass"}


def test_every_bucket_and_the_batch_hold_tuned_options():
    tab = json.load(open(tuning.TUNED))
    assert len(tab["buckets"]) == len(tuning.BUCKETS)
    for b, spec in zip(tab["buckets"], tuning.BUCKETS):
        assert b["n"] == spec["n"] and b["m"] == spec["m"]
        assert set(b["options"]) == KEYS, b
        assert b["report"]["evaluated"] > 1
        assert b["options"]["rows_near"] in (128, 256, 512)
    assert set(tuning.batch_options()) == KEYS


def test_unseen_inputs_get_the_options_of_their_bucket():
    tab = json.load(open(tuning.TUNED))["buckets"]
    for n, lo, hi in ((12_345, 10, 20), (77_777, 200, 260), (350_000, 60, 80),
                      (3_000_000, 300, 400), (500_000, 100, 120)):
        opts = tuning.options_for(n, lo, hi)
        q = tuning.bucket_of(n, (lo + hi) // 2, tab)
        b = tab[q]
        assert b["n"][0] <= n < b["n"][1] and b["m"][0] <= (lo + hi) // 2 < b["m"][1]
        assert opts == b["options"]
