"""Host logic of the split and sliced-layout planner, without a GPU.

`host_plan_check.cpp` links the library's host sources (CSR ingest,
partitioners, tile planner) with the host C++ compiler, plans the 7-point
Laplacian under each split, and decodes every stored entry from its slot the
way the sweep kernel does (row + shift, a relative or global column, or an
LDS position mapped back through the tile's footprint runs) against the
permuted matrix.  The tests check that program's verdict and the planner's
choices: the column format per split, the tile cost spread that picks the
launch grid, and the tile ranges of the eight XCDs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_02377_amd", "csrc")
SOURCES = ["host_plan.cpp", "host_partition.cpp", "host_csr.cpp", "host_graph.cpp"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not shutil.which("g++") or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("plan") / "host_plan_check")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(ROOT, "tests", "host_plan_check.cpp")] + [os.path.join(CSRC, f) for f in SOURCES]
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True)
    return exe


def run(exe, *args):
    p = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    tok = p.stdout.split()
    out = {"fmt": int(tok[1]), "ntiles": int(tok[3]), "slots": int(tok[5]), "spread": float(tok[7]),
           "xcd": [int(t) for t in tok[9:18]]}
    return out


@pytest.mark.parametrize("N,mode,P,sub,fmt", [(24, 1, 8, 2, 3), (24, 2, 8, 2, 4), (24, 3, 8, 2, 2), (32, 3, 64, 4, 2),
                                              (17, 1, 3, 2, 3), (17, 2, 5, 2, 4)])
def test_every_entry_decodes_from_its_slot(checker, N, mode, P, sub, fmt):
    r = run(checker, N, mode, P, sub)
    # band rows reach their columns through one shift per stencil neighbour
    # (a shift table; staged: LDS position minus row); substructuring's
    # interface tiles do not, and keep 16-bit tile-local columns
    assert r["fmt"] == fmt
    assert r["slots"] >= 7 * N ** 3 - 6 * N ** 2
    xcd = r["xcd"]
    assert xcd[0] == 0 and xcd[8] == r["ntiles"] and all(u <= v for u, v in zip(xcd, xcd[1:]))


@pytest.mark.parametrize("mode,layout,fmt", [(1, 1, 1), (1, 2, 0), (2, 1, 2), (3, 1, 2)])
def test_explicit_column_formats_decode(checker, mode, layout, fmt):
    # without shift tables: row-relative 16-bit columns (unstaged), 32-bit
    # global ones when asked, tile-local 16-bit LDS positions (staged)
    r = run(checker, 20, mode, 6, 2, layout)
    assert r["fmt"] == fmt


def test_tile_cost_spread_and_xcd_ranges(checker):
    jb = run(checker, 32, 1, 8, 2)
    jbo = run(checker, 32, 2, 8, 2)
    jss = run(checker, 32, 3, 64, 4)
    # alike band-row tiles: one resident round, equal tile counts per XCD
    for r in (jb, jbo):
        assert r["spread"] <= 1.25
        counts = [v - u for u, v in zip(r["xcd"], r["xcd"][1:])]
        assert max(counts) - min(counts) <= 1
    # substructuring: interface tiles gather many footprint runs
    assert jss["spread"] > 1.25
    counts = [v - u for u, v in zip(jss["xcd"], jss["xcd"][1:])]
    assert sum(counts) == jss["ntiles"] and min(counts) > 0


def random_csr(path, seed, n=3000):
    """A seeded random pattern with the diagonal, short local rows and some
    rows of 50-300 entries spread over all columns (wider than a 64-lane slot
    mask), written for the checker's --csr mode."""
    import numpy as np
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        if rng.random() < 0.05:
            c = rng.integers(0, n, int(rng.integers(50, 300)))
        else:
            c = i + rng.integers(-30, 31, int(rng.integers(0, 8)))
        c = np.unique(np.concatenate([c[(c >= 0) & (c < n)], [i]]))
        rows.append(c.astype(np.int32))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    with open(path, "wb") as f:
        f.write(np.array([n], np.int32).tobytes() + np.array([rp[-1]], np.int64).tobytes())
        f.write(rp.tobytes() + np.concatenate(rows).tobytes())


@pytest.mark.parametrize("mode,P,part", [(1, 3, 0), (2, 4, 0), (2, 5, 1), (3, 6, 0), (3, 4, 1)])
def test_random_patterns_with_rows_wider_than_a_slot_mask(checker, tmp_path, mode, P, part):
    # rows of hundreds of entries make slices wider than 64 slots (as wide as
    # the widest row): the split and every layout must plan and decode them
    path = str(tmp_path / "a.bin")
    random_csr(path, 17 + mode)
    p = subprocess.run([checker, "--csr", path, str(mode), str(P), str(part)], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    assert int(p.stdout.split()[1]) in (0, 1, 2, 3, 4)
