"""Launch planning on the host, no GPU: the large-graph BP kernel's message layout and the slot
kernel's message stride, both chosen from a model of the LDS banks (32 four-byte banks serving a
wavefront in two halves of 32 lanes).  A small C++ program (tests/host/plan_check.cpp) links the
built library and calls its planning functions on graphs written here."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2406_18655_amd.workloads import bivariate_bicycle, random_34_hgp, synthetic_dem

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2406_18655_amd")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    if not os.path.exists(os.path.join(PKG, "libqlsd.so")):
        pytest.skip("libqlsd.so not built (run __graft_entry__.build())")
    out = str(tmp_path_factory.mktemp("plan") / "plan_check")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(HERE, "host", "plan_check.cpp"), "-L", PKG, "-lqlsd", f"-Wl,-rpath,{PKG}", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _graph_file(tmp_path, H, name):
    H = np.asarray(H, dtype=np.uint8)
    rows, cols = np.nonzero(H)
    rp = np.zeros(H.shape[0] + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    p = tmp_path / name
    with open(p, "w") as f:
        f.write(f"{H.shape[0]} {H.shape[1]} {len(rows)}\n")
        f.write(" ".join(map(str, cols)) + "\n")
        f.write(" ".join(map(str, rp)) + "\n")
    return str(p)


def _run(checker, *args):
    r = subprocess.run([checker, *map(str, args)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    v = r.stdout.split()
    return {v[k]: float(v[k + 1]) for k in range(0, len(v), 2)}


def test_large_graph_layout_on_the_dem(checker, tmp_path):
    """The 936 x 8800 detector error model: every fault entry at its own word inside the layout,
    every check visiting exactly its own edges, the fault phase free of bank conflicts (groups of
    64 faults interleaved) and the check phase at most 1.65 modelled cycles per half-wavefront
    access (3.4 for the CSC order)."""
    code = synthetic_dem()
    res = _run(checker, "layout", _graph_file(tmp_path, code.H, "dem.txt"))
    assert res["consistent"] == 1
    assert code.H.sum() <= res["words"] < 32768          # padded only where a group mixes weights
    assert res["words"] <= code.H.sum() + 64 * 8
    assert res["fault"] == 1.0
    assert res["check"] <= 1.65


def test_large_graph_layout_on_two_column_weights(checker, tmp_path):
    """A hypergraph product of (3,4)-regular codes, whose columns weigh 3 or 4: in the weight order
    only one group of 64 faults straddles the two weights (at most 64 words of padding), and the
    last, partial group is laid out as a whole one (at most 64 times its weight)."""
    code = random_34_hgp(16, p=0.03)
    assert sorted(set(code.H.sum(axis=0).tolist())) == [3, 4]
    res = _run(checker, "layout", _graph_file(tmp_path, code.H, "hgp16.txt"))
    assert res["consistent"] == 1 and res["fault"] == 1.0
    assert code.H.sum() <= res["words"] <= code.H.sum() + 64 + 64 * 4


def test_slot_stride_on_bb144(checker, tmp_path):
    """[[144,12,12]] (432 edges) at its default 14 slots in 40 KB per workgroup: the model picks
    437 (the odd stride 433 measured 7 % slower for BP), and the block still fits."""
    code = bivariate_bicycle(p=0.05)
    res = _run(checker, "stride", _graph_file(tmp_path, code.H, "bb.txt"), 14, 40960)
    assert res["stride"] == 437
    assert res["bytes"] <= 40960


@pytest.mark.parametrize("S,budget", [(20, 162816), (4, 40960)])
def test_slot_stride_stays_in_budget(checker, tmp_path, S, budget):
    """Any chosen stride lies in [nnz, nnz + 63] and keeps the block within its budget."""
    code = random_34_hgp(16, p=0.03)
    E = int(code.H.sum())
    res = _run(checker, "stride", _graph_file(tmp_path, code.H, "hgp16.txt"), S, budget)
    assert E <= res["stride"] < E + 64
    assert res["bytes"] <= budget
