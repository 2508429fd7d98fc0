"""Host-side pieces of the benchmark: the counter summaries it reads (HBM
bytes per launch, guarded by a hash of the kernel's sources; VALU busy per
kernel) and the rule that labels a kernel's bound from its own counters."""
import hashlib
import os

import pytest

import bench


@pytest.fixture
def fake_tree(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1710_08314_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "a.hip").write_text("kernel a\n")
    (csrc / "b.hip").write_text("kernel b\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"ka": "ta.md", "kb": "tb.md"})
    monkeypatch.setattr(bench, "KERNEL_SOURCES", {"ka": ["a.hip"], "kb": ["b.hip"]})
    monkeypatch.setattr(bench, "ISSUE_FILE", "issue.md")
    return tmp_path


def _summary(root, name, sources, nbytes):
    h = hashlib.sha256()
    for f in sources:
        h.update((root / "paper_1710_08314_amd" / "csrc" / f).read_bytes())
    (root / "profiles" / name).write_text(
        "# summary\n\n- kernel: `x`\n"
        f"- source_sha256: `{h.hexdigest()[:16]}`\n- traffic_bytes_per_launch: `{nbytes}`\n")


def _issue(root, rows):
    lines = ["| kernel | VGPR | LDS | VALU | SALU | LDS instr | mean ms / launch | VALU busy | LDS GB/s | c |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for k, ms, busy in rows:
        lines.append(f"| `{k}` | 64 | 0 | 1 | 1 | 1 | {ms} | {busy}% | 1.0 | 0.0 |")
    (root / "profiles" / "issue.md").write_text("\n".join(lines) + "\n")


def test_traffic_read_while_sources_match(fake_tree):
    _summary(fake_tree, "ta.md", ["a.hip"], 1234)
    _summary(fake_tree, "tb.md", ["b.hip"], 66)
    assert bench.measured_traffic("ka") == 1234
    assert bench.measured_traffic("ka + kb") == 1300
    # a changed source voids its figure, and a tier's sum with it
    (fake_tree / "paper_1710_08314_amd" / "csrc" / "b.hip").write_text("kernel b, edited\n")
    assert bench.measured_traffic("kb") is None
    assert bench.measured_traffic("ka + kb") is None
    assert bench.measured_traffic("kc") is None


def test_valu_busy_time_weighted(fake_tree):
    _summary(fake_tree, "ta.md", ["a.hip"], 1)
    _summary(fake_tree, "tb.md", ["b.hip"], 1)
    _issue(fake_tree, [("ka", 3.0, 50.0), ("kb", 1.0, 10.0)])
    assert bench.measured_valu_busy("ka") == pytest.approx(0.5)
    assert bench.measured_valu_busy("ka + kb") == pytest.approx((3.0 * 0.5 + 1.0 * 0.1) / 4.0)
    # no traffic summary for the sources as they are: no issue figure either
    (fake_tree / "paper_1710_08314_amd" / "csrc" / "a.hip").write_text("changed\n")
    assert bench.measured_valu_busy("ka") is None


def test_bound_from_counters():
    # the SC stage's counters: 15% of the HBM peak, VALU busy 54%: issue-bound
    assert bench.tier_bound(0.145, 0.54, 0.079) == "alu"
    # a kernel streaming at 61% of the HBM peak with its VALU half idle
    assert bench.tier_bound(0.61, 0.43, 0.04) == "hbm"
    # no counters: the algorithmic-op fraction stands in for issue
    assert bench.tier_bound(None, None, 0.05) == "alu"
    assert bench.tier_bound(0.2, None, 0.05) == "hbm"
