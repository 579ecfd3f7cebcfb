"""The committed rocprofv3 summaries agree with what bench.py reports from them.

* every command a summary gives runs committed files only (the repository's
  bench.py or a module of the package), with the program directly after
  ``--`` and counter passes that stay within one run's hardware limits;
* the traffic summaries hold the same per-dispatch FETCH_SIZE / WRITE_SIZE
  means, kernel name and source SHA-256 as the tables bench.py scales into
  ``roofline.traffic``, so a re-taken counter run cannot be reported from a
  stale table or the reverse.
"""
from __future__ import annotations

import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
if not os.path.isdir(PROFILES):   # a copy of the tree without the summaries
    pytest.skip("profiles/ is not present", allow_module_level=True)


def _summaries():
    return sorted(f for f in os.listdir(PROFILES) if f.endswith((".md", ".txt")))


def _commands(text: str):
    cmds, inside = [], False
    for line in text.splitlines():
        if line.startswith("```"):
            inside = not inside
            continue
        if inside and line.startswith("rocprofv3"):
            cmds.append(line.split())
    return cmds


@pytest.mark.parametrize("name", _summaries())
def test_profile_commands_run_committed_files(name):
    text = open(os.path.join(PROFILES, name)).read()
    assert "round" not in name.lower()
    cmds = _commands(text)
    assert cmds, f"{name} gives no rocprofv3 command"
    for argv in cmds:
        prog = argv[argv.index("--") + 1:]
        assert prog[0] in ("python", "python3"), argv
        prog = [prog[0]] + [x for x in prog[1:] if x != "-u"]  # unbuffered output changes nothing run
        if prog[1] == "-m":
            path = os.path.join(ROOT, *prog[2].split(".")) + ".py"
        else:
            path = os.path.join(ROOT, prog[1])
        assert os.path.isfile(path), f"{name}: {path} is not in the repository"
        assert "_work" not in " ".join(argv)
        if "--pmc" in argv:
            # counters go in runs of their own, without trace domains
            assert not {"--kernel-trace", "--stats", "-s", "--sys-trace", "-r",
                        "--runtime-trace"} & set(argv), argv
            counters = argv[argv.index("--pmc") + 1:argv.index("-d")]
            sq = [c for c in counters if c.startswith("SQ_")]
            tcc = [c for c in counters if c.startswith("TCC_") or c in ("FETCH_SIZE", "WRITE_SIZE")]
            assert len(sq) <= 8 and len(tcc) <= 2, argv


def _traffic_rows(text: str):
    sha = re.search(r"\b([0-9a-f]{64})\b", text).group(1)
    rows = re.findall(r"^\| `(k_stage[^`]*)` \| (\d+) \| ([\d.]+) \| ([\d.]+) \|", text, re.M)
    return sha, {k: (float(fe), float(wr)) for k, _, fe, wr in rows}


@pytest.mark.parametrize("name,table,K", [
    ("k_stage_mfma_q3_large_single_traffic.md", bench.MEASURED_TRAFFIC, None),
    ("k_stage_mfma_q3_fp64_large_single_traffic.md", bench.MEASURED_TRAFFIC_FP64, None),
    ("k_stage2d_p3_trap_disk_traffic.md", bench.MEASURED_TRAFFIC_2D, None),
    ("k_stage_mfma_q2_scatterer.md", bench.MEASURED_TRAFFIC_Q2, 1572864),
    ("k_stage_mfma_q2_batched_all_active.md", bench.MEASURED_TRAFFIC_Q2, 64 * 10368),
])
def test_traffic_summary_matches_bench_table(name, table, K):
    """K (when given) selects the table rows that the summary covers."""
    sha, rows = _traffic_rows(open(os.path.join(PROFILES, name)).read())
    tables = table if isinstance(table, list) else [table]
    tables = [t for t in tables if K is None or t["K"] == K]
    assert len(rows) == len(tables)
    for t in tables:
        assert sha == t["kernels_sha256"]
        assert rows[t["kernel"]] == (t["fetch_kib"], t["write_kib"])


@pytest.mark.parametrize("table,source", [
    (bench.MEASURED_TRAFFIC, "kernels.hip"),
    (bench.MEASURED_TRAFFIC_FP64, "kernels.hip"),
    (bench.MEASURED_TRAFFIC_Q2, "kernels.hip"),
    (bench.MEASURED_TRAFFIC_2D, "kernels2d.hip"),
])
def test_traffic_tables_match_the_current_kernel_source(table, source):
    """Every counter table belongs to the kernel source in the tree: a table
    left behind by a change of the source would make bench.py report no
    traffic (it checks the same digest at run time)."""
    import hashlib
    path = os.path.join(ROOT, "paper_2106_02858_amd", "csrc", source)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    for t in (table if isinstance(table, list) else [table]):
        assert t["kernels_sha256"] == digest, (source, t["kernel"])
