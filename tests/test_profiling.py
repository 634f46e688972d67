"""Host logic of the profile summaries: a stage line written by the traffic
summary is read back by the benchmark, and only while the kernel's sources
are unchanged."""
import os

from paper_2109_00214_amd import profiling as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stage_line_round_trip(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("# header\n" + PR.stage_line("push", 2.0e8, 1.5e8, 3.0e6) + "\n")
    got = PR.read_traffic(str(p))
    assert abs(got["push"] - 350.0e6 / 3.0e6) < 0.01


def test_stale_digest_is_ignored(tmp_path):
    line = PR.stage_line("push", 2.0e8, 1.5e8, 3.0e6).split()
    line[-1] = "0" * 16
    p = tmp_path / "t.txt"
    p.write_text(" ".join(line) + "\n")
    assert PR.read_traffic(str(p)) == {}


def test_committed_summaries_have_stage_lines():
    """The benchmark's summary carries the push line, the deposit run's
    summary the deposit line."""
    for name, stage in (("hbm_traffic_paper_256x512.txt", "push"),
                        ("hbm_traffic_deposit_paper_256x512.txt", "deposit")):
        path = os.path.join(ROOT, "profiles", name)
        stages = [l.split() for l in open(path) if l.startswith("stage ")]
        assert stage in {w[1] for w in stages}, name
        assert all(len(w) == 10 and w[1] in PR.STAGE_KERNELS for w in stages), name
