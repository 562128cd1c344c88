"""Host logic of bench.py (no GPU): the stored-form byte accounting behind
the roofline, the kernel named for each format, the rule that counter
traffic is reported only for the kernel source it was taken on, and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench
from paper_1701_03989_amd import sscg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_form_bytes_per_format():
    n, stored = 1000, 64 * 16 * 7  # 16 slices, widths 7
    nsl = 16
    # slice-diagonal: a 16-bit code per row (padded to whole slices) and per
    # slice its count, 8 distances and 4-entry table; the pair and value bits
    # change nothing stored
    sd = 2.0 * 64 * nsl + (4 + 4 * 8 + 32) * nsl
    for extra in (0, sscg.FMT_SDPAIR, sscg.FMT_SDPAIR | sscg.FMT_SDVAL, sscg.FMT_SDVAL):
        assert bench.form_bytes(sscg.FMT_SDIA | extra, stored, n) == sd
    # value index + 16-bit offset; value + 16-bit offset; value + 32-bit index
    assert bench.form_bytes(sscg.FMT_COL16 | sscg.FMT_VTAB, stored, n) == 3 * stored + 44 * nsl
    assert bench.form_bytes(sscg.FMT_COL16, stored, n) == 10 * stored + 12 * nsl
    assert bench.form_bytes(0, stored, n) == 12 * stored + 12 * nsl


def test_form_name_follows_the_format_bits():
    sd = sscg.FMT_SDIA | sscg.FMT_COL16 | sscg.FMT_VTAB
    assert bench.form_name(sd | sscg.FMT_SDPAIR | sscg.FMT_SDVAL).startswith("k_mpk_sdp ")
    assert bench.form_name(sd | sscg.FMT_SDPAIR).startswith("k_mpk_sdp ")
    assert "slice-diagonal" in bench.form_name(sd) and bench.form_name(sd).startswith("k_mpk ")
    assert "value tables" in bench.form_name(sscg.FMT_COL16 | sscg.FMT_VTAB)
    assert "16-bit" in bench.form_name(sscg.FMT_COL16)
    assert "32-bit" in bench.form_name(0)


def test_traffic_is_reported_only_for_the_source_it_was_taken_on(tmp_path):
    ok = {"source_sha256_16": bench.source_hash(bench.MPK_SOURCES),
          "hbm_bytes_per_launch": 1.25e8, "launches": 3}
    p = tmp_path / "summary.md"
    p.write_text("# summary\n\n" + json.dumps(ok) + "\n")
    assert bench.traffic_from_profile(str(p)) == 1.25e8
    stale = dict(ok, source_sha256_16="0" * 16)
    p.write_text("# summary\n\n" + json.dumps(stale) + "\n")
    assert bench.traffic_from_profile(str(p)) is None
    p.write_text("# summary without the machine-readable line\n")
    assert bench.traffic_from_profile(str(p)) is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""
