"""Stage breakdown of the shard build kernel (k_build) on the benchmark's
VFilter workload, from the stage clocks of the profiling build of the
library.  Run with that build selected:

    python -m paper_2503_18397_amd.build --stage-clocks
    VF_LIBRARY=$PWD/paper_2503_18397_amd/libvf_stages.so \\
        python -m paper_2503_18397_amd.stage_profile [--log2n 27] [--b 8]

Prints one JSON object: the build's time, and per workgroup and per item
the time of the peeling, elimination and assignment stages, then per
32-column word of the elimination the phases of the searching wavefront
and of an emitting one (microseconds).  The clocks add a few atomics per
word, so the totals run a little above the plain library's."""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=27)
    ap.add_argument("--b", type=int, default=8)
    ap.add_argument("--eps", type=float, default=0.0175)
    ap.add_argument("--data-seed", type=int, default=2027)
    ap.add_argument("--repeat", type=int, default=2)
    args = ap.parse_args()

    import torch

    import paper_2503_18397_amd as vf
    import synthetic as S
    if not vf.LIB_PATH.endswith("libvf_stages.so"):
        sys.exit("select the stage-clock build: VF_LIBRARY=.../libvf_stages.so")
    keys = S.member_keys(1 << args.log2n, args.data_seed, device="cuda:0")
    out = None
    for _ in range(args.repeat):  # the last run is reported
        vf.vf_stage_clocks(reset=True)
        st = vf.Structure.build(keys, None, b=args.b, eps=args.eps)
        torch.cuda.synchronize()
        info = st.info
        raw = vf.vf_stage_clocks().astype(np.float64)
        st.free()
        used = raw[:, 7] > 0
        raw = raw[used]
        us = raw / 100.0  # tick slots: 100 MHz ticks -> microseconds

        def per(t, n):
            return round(float(us[:, t].sum() / max(raw[:, n].sum(), 1)) / 1e3, 3)

        names = ("returns_and_entering_rows", "compaction", "pivot_search", "row_updates",
                 "flags", "barrier")
        ph = {}
        for who, o in (("searching_wavefront", 8), ("emitting_wavefront", 16)):
            w = max(raw[:, o + 6].sum(), 1)
            ph[who] = {k: round(float(us[:, o + i].sum() / w), 3) for i, k in enumerate(names)}
            ph[who]["words_per_workgroup"] = round(float(w / len(raw)), 1)
        e = ph["emitting_wavefront"]
        ph["emitting_wavefront"] = {"emission": e["compaction"],
                                    "wait_for_batch_and_row_updates": e["pivot_search"],
                                    "barrier": e["barrier"],
                                    "words_per_workgroup": e["words_per_workgroup"]}
        att = max(raw[:, 30].sum(), 1)
        pnames = ("edges_and_cleared_state", "incidence", "first_frontier", "rounds",
                  "core_grouping", "duplicate_row_check")
        peel = {k: round(float(us[:, 24 + i].sum() / att), 1) for i, k in enumerate(pnames)}
        peel["attempts"] = int(att)
        peel["rounds_per_attempt"] = round(float(raw[:, 31].sum() / att), 1)
        out = {
            "workload": f"VFilter b={args.b}, n=2^{args.log2n}, eps={args.eps}",
            "S": info["S"], "M": info["M"], "sigma": info["sigma"],
            "ms_build": round(info["ms_build"], 3), "failed_attempts": info["n_failures"],
            "workgroups": int(used.sum()),
            "per_workgroup_ms": {
                "total": round(float(us[:, 7].mean()) / 1e3, 3),
                "max_total": round(float(us[:, 7].max()) / 1e3, 3),
                "first_item_all_wavefronts": round(float(us[:, 6].mean()) / 1e3, 3),
                "peeling_wavefront": round(float(us[:, 0].mean()) / 1e3, 3),
                "elimination": round(float(us[:, 2].mean()) / 1e3, 3),
                "assignment": round(float(us[:, 4].mean()) / 1e3, 3)},
            "after_last_elimination_ms": {
                "mean": round(float((us[:, 7] - us[:, 23]).mean()) / 1e3, 3),
                "of_the_slowest_workgroup": round(float(
                    (us[:, 7] - us[:, 23])[int(us[:, 7].argmax())]) / 1e3, 3)},
            "per_item_ms": {"peel": per(0, 1), "elimination": per(2, 3),
                            "assignment": per(4, 5), "of_which_back_substitution": per(15, 5)},
            "per_word_us": ph,
            "peel_per_attempt_us": peel,
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
