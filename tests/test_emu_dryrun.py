"""bench.py and __graft_entry__.smoke() run end to end on the CPU against the emulated library
(tests/hipemu/dryrun.py: a numpy stand-in for torch, the package bound to the emulated build),
at toy sizes.  This checks the scripts' own logic -- every leg, the JSON contract, the label
comparisons inside them -- without a GPU; the figures are the emulator's and mean nothing."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRY = os.path.join(HERE, "hipemu", "dryrun.py")
ROOT = os.path.dirname(HERE)

pytest.importorskip("hipemu")


def run(args, timeout):
    proc = subprocess.run([sys.executable, DRY] + args, cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, timeout=timeout)
    assert proc.returncode == 0, proc.stderr[-3000:]
    return proc


def test_smoke_runs():
    assert "smoke ok" in run(["smoke"], 300).stdout


@pytest.mark.slow
def test_bench_json_contract():
    proc = run(["bench", "--workload", "small", "--steps", "2", "--warmup", "2", "--secondary", "",
                "--tune-knobs", "round0,round0_sort,row_pairs,tail", "--set", "tail=2,radix_form=2",
                "--variant-steps", "1", "--batch-graphs", "12", "--batch-log2-max", "9", "--batch-steps", "1",
                "--serve-requests", "6", "--serve-warmup", "2", "--serve-pool", "3", "--serve-log2-max", "12",
                "--serve-loads", "1.0", "--serve-budget-gib", "1"],
               900)
    lines = [x for x in proc.stdout.splitlines() if x.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["config"]["workload"].startswith("G(n=65,536")
    assert d["config"]["tuning"]["tail"] == 2 and d["config"]["tuning"]["radix_form"] == 2   # --set, untuned
    assert d["tuner_rejected"] == []
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["kernel"].startswith("a") and r["frac"] == round(r["achieved"] / 8000.0, 4)
    sr = d["step_rooflines"]
    assert r["kernel"] in sr and {"a2_one_hop", "a4_relabel", "a5_dedup"} <= set(sr)
    assert all(v["ms_per_solve"] >= 0 for v in sr.values())
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 1 and "of" in c["host"] and "union_find" in c
    assert all(v["canonical_labels_identical"] for v in d["variants"].values())
    assert set(d["variants"]) == {"tree", "one_hop", "uf_finish", "merge_to_large"}
    assert d["batched"]["labels_identical_to_sequential"] and d["batched"]["tuner_rejected"] == []
    assert d["serving"]["labels_identical_to_solo"]
    assert d["serving"]["requests"] == 6 and d["serving"]["warmup_requests"] == 2 and d["serving"]["pool_graphs"] == 3
    # more than one GPU is refused with a message
    proc = subprocess.run([sys.executable, DRY, "bench", "--gpus", "2"], cwd=ROOT, stdout=subprocess.PIPE,
                          stderr=subprocess.PIPE, text=True, timeout=120)
    assert proc.returncode == 2 and "one GPU" in proc.stderr
