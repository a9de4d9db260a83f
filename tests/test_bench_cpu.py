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
