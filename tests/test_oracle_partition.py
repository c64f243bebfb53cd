"""Pins of the oracle partitioner: the paper's dependency table, hand-derived
closed forms of halo and interface sizes, and brute-force definitions on
small grids.  CPU only."""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from oracle import partition as OP
from oracle import ref
from paper_2112_02377_amd import workloads as W


def tab_dep():
    g = read_golden("tab_dep.txt")
    pairs = [tuple(int(v) - 1 for v in t.split("/")) for t in g["PATTERN"][0]]
    n = 1 + max(max(p) for p in pairs)
    rows = [[] for _ in range(n)]
    for r, c in pairs:
        rows[r].append(c)
    rp = np.zeros(n + 1, np.int32)
    ci = []
    for r in range(n):
        ci += sorted(rows[r])
        rp[r + 1] = len(ci)
    P = int(g["NPROC"][0][0])

    def lists(key):
        out = {}
        for t in g[key]:
            a, b = int(t[0]) - 1, int(t[1]) - 1
            out[(a, b)] = [int(v) - 1 for v in t[3:]]
        return out
    return rp, np.array(ci, np.int32), P, lists("RECV"), lists("SEND")


def test_band_row_dependency_lists_of_the_paper_example():
    rp, ci, P, recv, send = tab_dep()
    assert list(OP.band_bounds(10, P)) == [0, 3, 6, 10]
    part = OP.partition(rp, ci, OP.JBO, P)
    got = {}
    for p in range(P):
        for idx in part["recv_idx"][part["recv_ptr"][p]:part["recv_ptr"][p + 1]]:
            got.setdefault((p, int(part["owner"][idx])), []).append(int(idx))
    assert got == recv
    sptr, sdest, sidx = OP.send_lists(part["recv_ptr"], part["recv_idx"], part["owner"], P)
    gots = {}
    for q in range(P):
        for d, i in zip(sdest[sptr[q]:sptr[q + 1]], sidx[sptr[q]:sptr[q + 1]]):
            gots.setdefault((q, int(d)), []).append(int(i))
    assert gots == send
    # naive band-row: no lists, identity order
    jb = OP.partition(rp, ci, OP.JB, P)
    assert len(jb["recv_idx"]) == 0 and np.array_equal(jb["perm"], np.arange(10))


def test_jbo_halo_closed_form_small():
    # N=20, 4 bands of 5 planes: each inner band boundary costs one plane
    # (N^2 = 400 nodes) in each direction: H = 2 * 3 * 400
    s = W.laplace7(20)
    part = OP.partition(s.row_ptr, s.col_idx, OP.JBO, 4)
    assert len(part["recv_idx"]) == 2400


def brute_recv(rp, ci, owner, P):
    out = [set() for _ in range(P)]
    n = len(rp) - 1
    for r in range(n):
        for p in range(rp[r], rp[r + 1]):
            c = int(ci[p])
            if owner[c] != owner[r]:
                out[owner[r]].add(c)
    lst = []
    for p in range(P):
        lst += sorted(out[p], key=lambda c: (owner[c], c))
    return lst


@pytest.mark.parametrize("grid,sub,P", [((6, 5, 4), (2, 2, 2), 3), ((7, 6, 5), (3, 2, 2), 12),
                                        ((5, 5, 5), (2, 1, 3), 2)])
def test_substructuring_matches_brute_force_definitions(grid, sub, P):
    nx, ny, nz = grid
    rp, ci, _ = W.stencil7_pattern(nx, ny, nz)
    n = nx * ny * nz
    part = OP.partition(rp, ci, OP.JSS, P, grid=grid, sub_grid=sub)
    sx, sy, sz = sub
    # block of a coordinate by the floor band rule
    def blk(c, m, s_):
        return max(b for b in range(s_) if (b * m) // s_ <= c)
    subid = np.zeros(n, int)
    for r in range(n):
        i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
        subid[r] = blk(i, nx, sx) + sx * (blk(j, ny, sy) + sy * blk(k, nz, sz))
    assert np.array_equal(part["sub"], subid)
    # interface: a neighbour (either direction) in another subdomain
    ifc = np.zeros(n, bool)
    for r in range(n):
        for p in range(rp[r], rp[r + 1]):
            c = ci[p]
            if c != r and subid[c] != subid[r]:
                ifc[r] = ifc[c] = True
    S = sx * sy * sz
    order = [r for s_ in range(S) for r in range(n) if not ifc[r] and subid[r] == s_]
    order += sorted([r for r in range(n) if ifc[r]], key=lambda r: (subid[r], r))
    assert list(part["perm"]) == order
    n_int = int((~ifc).sum())
    assert part["n_interior"] == n_int
    sub_int_ptr = part["bounds"][:S + 1]
    sub_ifc_ptr = part["bounds"][S + 1:2 * S + 2]
    part_sub_ptr = part["bounds"][2 * S + 2:]
    for s_ in range(S):
        assert sub_int_ptr[s_ + 1] - sub_int_ptr[s_] == sum(1 for r in range(n) if not ifc[r] and subid[r] == s_)
        assert sub_ifc_ptr[s_ + 1] - sub_ifc_ptr[s_] == sum(1 for r in range(n) if ifc[r] and subid[r] == s_)
    assert list(part_sub_ptr) == [(q * S) // P for q in range(P + 1)]
    # receive lists in the new numbering, by brute force on the permuted matrix
    nrp, nci, _ = OP.permute_csr(rp, ci, None, part["perm"])
    owner = part["owner"]
    assert list(part["recv_idx"]) == brute_recv(nrp, nci, owner, P)
    # every received entry is an interface node (interiors never cross)
    assert np.all(part["recv_idx"] >= n_int)


def test_permuted_system_iterates_are_a_permutation_of_plain_iterates():
    # synchronous iterations do not depend on the ordering (paper: same
    # iteration counts for every split); rounding differs only in row sums
    s = W.laplace7(8, workload=1)
    part = OP.partition(s.row_ptr, s.col_idx, OP.JSS, 4, grid=s.grid, sub_grid=(2, 2, 2))
    perm = part["perm"]
    nrp, nci, nv = OP.permute_csr(s.row_ptr, s.col_idx, s.vals, perm)
    _, x, h = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 60)
    _, xp, hp = ref.sweeps(nrp, nci, nv, s.b[0][perm], 60)
    assert np.allclose(xp, x[perm], rtol=0, atol=1e-12 * np.abs(x).max())
    assert np.allclose(hp, h, rtol=1e-12)
    st1, _, k1, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 5000)
    st2, _, k2, _ = ref.solve(nrp, nci, nv, s.b[0][perm], 1e-8, 5000)
    assert st1 == st2 == ref.OK and k1 == k2


@pytest.mark.slow
def test_closed_forms_at_128_cubed():
    """Hand-derived sizes for the 128^3 7-point grid and 64 parts.

    JBO: 64 bands of 2 planes; 63 inner boundaries, each costing one 128^2
    plane in both directions: H = 2*63*128^2.
    JSS with 8^3 subdomains of 16^3: along each axis the 7 inner block
    boundaries each put 2 node layers on the interface, so interior =
    (128-14)^3.  Eight consecutive ids (x fastest) form one part = a 128x16x16
    beam; beams touch across y and z faces of 128*16 nodes, 2*8*7 adjacent
    pairs, each received in both directions: H = 2*112*2048.
    JSS with 4^3 subdomains of 32^3 (one per part): interior = (128-6)^3;
    3*4*4*3 = 144 adjacent pairs of 32^2 faces, both directions:
    H = 2*144*1024.
    """
    N = 128
    rp, ci, _ = W.stencil7_pattern(N, N, N)
    jbo = OP.partition(rp, ci, OP.JBO, 64)
    assert len(jbo["recv_idx"]) == 2 * 63 * N * N == 2_064_384
    assert 63 * N ** 3 == 132_120_576     # the naive gather volume (whole x minus own band)
    j8 = OP.partition(rp, ci, OP.JSS, 64, grid=(N, N, N), sub_grid=(8, 8, 8))
    assert j8["n_interior"] == 114 ** 3 == 1_481_544
    assert N ** 3 - j8["n_interior"] == 615_608
    assert len(j8["recv_idx"]) == 2 * (2 * 8 * 7) * (128 * 16) == 458_752
    j4 = OP.partition(rp, ci, OP.JSS, 64, grid=(N, N, N), sub_grid=(4, 4, 4))
    assert j4["n_interior"] == 122 ** 3 == 1_815_848
    assert len(j4["recv_idx"]) == 2 * 144 * 1024 == 294_912


def test_permutations_are_permutations():
    for grid, sub, P in [((9, 7, 5), (3, 1, 2), 5), ((4, 4, 4), (1, 1, 1), 1)]:
        rp, ci, _ = W.stencil7_pattern(*grid)
        n = int(np.prod(grid))
        for mode in (OP.JB, OP.JBO, OP.JSS):
            part = OP.partition(rp, ci, mode, P, grid=grid, sub_grid=sub)
            assert np.array_equal(np.sort(part["perm"]), np.arange(n))
    # without a grid, substructuring falls back to contiguous row blocks
    rp, ci, _ = W.stencil7_pattern(6, 6, 6)
    part = OP.partition(rp, ci, OP.JSS, 3, grid=None, sub_grid=(6, 1, 1))
    assert np.array_equal(part["sub"], OP.band_of(np.arange(216), OP.band_bounds(216, 6)))
    assert list(itertools.islice(part["bounds"][-4:], 4)) == [0, 2, 4, 6]
