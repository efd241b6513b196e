"""Host-side checks of bench.py's bookkeeping (no GPU): the counter summary committed for the
headline step names every kernel that the timed records map to, so a renamed kernel cannot
silently turn the reported HBM traffic into null."""

import glob
import json
import os

import bench


def _summaries():
    return sorted(glob.glob(os.path.join(bench.PROFILES, "hbm_traffic_allknn_1M_d128_T*_bf16x3.md")))


def test_a_headline_traffic_summary_is_committed():
    assert _summaries(), "no counter summary of the headline step under profiles/"


def test_every_record_kernel_is_in_the_summary():
    for path in _summaries():
        with open(path) as fh:
            table = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        names = table["kernels"].keys()
        for record, pat in bench.RECORD_KERNEL.items():
            pat = pat.format(p=bench.PREC_INDEX["bf16x3"])
            prefix = pat.endswith("<") or pat.endswith("true")
            assert any(k == pat or (prefix and k.startswith(pat)) for k in names), (path, record, pat)


def test_summary_file_follows_the_tree_count():
    T = int(os.path.basename(_summaries()[-1]).split("_T")[1].split("_")[0])
    assert bench.traffic_file(T) == _summaries()[-1]
    assert bench._traffic_table(T + 1000) is None
