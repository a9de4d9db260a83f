"""Host-side arithmetic of the benchmark: the algorithmic byte counts behind
the roofline figures, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_colored_bytes_count_records_and_face_data():
    # 2D, p = 2: records of 4 x 6 doubles; an interior face moves both sides'
    # DOF record read and RHS record read + write, a wall face one side
    rec = 4 * 6
    one_interior = bench.algorithmic_bytes(1, 1, rec, 8, 2)
    one_wall = bench.algorithmic_bytes(1, 0, rec, 8, 2)
    face = (2 + 3) * 8 + 8 + 2
    assert one_interior == 2 * 3 * rec * 8 + face == 1202
    assert one_wall == 3 * rec * 8 + face
    # the headline mesh: 1,497,218 faces, 3,520 on walls
    assert bench.algorithmic_bytes(1_497_218, 1_497_218 - 3_520, rec, 8, 2) == 1_797_628_516


def test_compact_bytes_are_fewer_than_colored_on_the_headline_mesh():
    E, nb, K = 1_497_218, 3_520, 996_972
    colored = bench.algorithmic_bytes(E, E - nb, 24, 8, 2)
    compact = bench.compact_bytes(E, E - nb, K, 4, 6, 3, 3, 8, 2)
    # face pass: both records read, face data, one record of 3 x 4 + 1 doubles written;
    # element pass: slots, sqrt(det J), the face records of every side, RHS read + write
    frec = (3 * 4 + 1) * 8
    face = (2 * E - nb) * 192 + E * ((2 + 3) * 8 + 8 + 2 + frec)
    elem = K * (3 * 4 + 8 + 2 * 192) + (2 * E - nb) * frec
    assert compact == face + elem
    assert compact < colored


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("fam", sorted(bench.SWEEP_SIDES))
def test_sweep_sizes_follow_the_paper_tables(fam):
    import json

    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    sides = [s for s, _ in golden["figure9_conflicts"][fam]]
    assert bench.SWEEP_SIDES[fam] == tuple(sides)


@pytest.mark.parametrize("profile,n_face,n_bnd,rec,dim,n_colors", [
    ("surface_colored_team_prefetch_delaunay996k_p2_f64.md", 1_497_218, 3_520, 4 * 6, 2, 3),
    ("surface_colored_mode_team_kuhn64_tets_p1_f64.md", 3_145_728, 0, 5 * 4, 3, 4),
    ("surface_colored_team_prefetch_quads1024_p2_f64.md", 2_097_152, 0, 4 * 9, 2, 4),
])
def test_profiles_quote_the_benchmark_byte_counts(profile, n_face, n_bnd, rec, dim, n_colors):
    """The algorithmic bytes per launch that each colored-pass profile divides
    its counters by are the benchmark's own count for that workload."""
    import re

    text = open(os.path.join(ROOT, "profiles", profile)).read()
    per_launch = bench.algorithmic_bytes(n_face, n_face - n_bnd, rec, 8, dim) // n_colors
    quoted = re.search(r"Algorithmic bytes per launch: ([0-9,]+) B", text)
    assert quoted is not None
    assert int(quoted.group(1).replace(",", "")) == per_launch


def test_profiled_traffic_matches_the_profile_of_the_committed_kernels():
    """bench.py reports the counter traffic only for the configuration and
    kernel sources the profile was taken with."""
    import hashlib
    import re
    import types

    args = types.SimpleNamespace(workload="delaunay", layout="paired", seed=2, points=500_000, p=2, tet_n=64)
    launch = {"form": "default", "block": 256, "xcd_remap": False}
    text = open(bench.PROFILES["delaunay"]).read()
    sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in bench.KERNEL_SOURCES)).hexdigest()[:16]
    if re.search(r"kernel_source_sha256_16: ([0-9a-f]{16})", text).group(1) != sha:
        pytest.skip("the kernel sources changed since the profile was taken")
    traffic = int(re.search(r"traffic_bytes_per_launch: (\d+)", text).group(1))
    assert bench.profiled_traffic(args, launch) == traffic
    # another layout, launch or size: no figure
    assert bench.profiled_traffic(types.SimpleNamespace(**{**vars(args), "layout": "paper"}), launch) is None
    assert bench.profiled_traffic(args, {**launch, "xcd_remap": True}) is None
    assert bench.profiled_traffic(types.SimpleNamespace(**{**vars(args), "points": 20_000}), launch) is None
