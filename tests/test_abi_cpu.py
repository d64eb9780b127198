"""C-ABI checks that need no GPU.

* libbfmf.so loads and exports every function include/bfmf.h declares.
* The C++ analysis (host-only handle) reproduces the oracle's ordering,
  assembly tree, update sets, extend-add maps and separator trees bit-exactly.
* Error paths: malformed CSR, non-finite values, calls out of order.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from workloads import helmholtz_7pt
from workloads.maxwell import yee_curlcurl
from oracle import nd
from oracle.symbolic import symbolic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
bfmf = pytest.importorskip("paper_2007_00202_amd.bfmf")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bfmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfmf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bfmf.LIB_PATH)
    names = declared_functions()
    assert "bfmf_analyze" in names and "bfmf_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(bfmf.EXPORTED)


def _compare(h, od, sym):
    s = bfmf.bfmf_get_symbolic(h)
    assert np.array_equal(s["perm"], od.perm)
    assert np.array_equal(s["sbeg"], od.sbeg) and np.array_equal(s["send"], od.send)
    assert np.array_equal(s["parent"], od.parent)
    kids = [list(s["child_list"][s["child_ptr"][f]:s["child_ptr"][f + 1]]) for f in range(od.nfronts)]
    assert kids == [list(c) for c in od.children]
    for f in range(od.nfronts):
        assert np.array_equal(s["iu"][s["iu_ptr"][f]:s["iu_ptr"][f + 1]], sym.Iu[f])
        assert np.array_equal(s["map"][s["iu_ptr"][f]:s["iu_ptr"][f + 1]], sym.maps[f])
        nodes = s["sep_nodes"][s["sep_ptr"][f]:s["sep_ptr"][f + 1]]
        assert nodes.tolist() == [list(t) for t in od.septree[f]]
    return s


@pytest.mark.parametrize("dims,leaf,sl", [((6, 6, 6), 27, 8), ((8, 8, 8), 64, 16), ((7, 5, 9), 20, 16),
                                          ((11, 11, 1), 10, 3), ((24, 24, 24), 512, 64)])
def test_cpp_analysis_matches_oracle_grid(dims, leaf, sl):
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    h = bfmf.bfmf_create(-1)
    try:
        bfmf.bfmf_analyze(h, rp, ci, v, dims=dims, leaf_max=leaf, sep_leaf=sl)
        od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=sl)
        sym = symbolic(rp, ci, od)
        s = _compare(h, od, sym)
        lv = np.zeros(od.nfronts, np.int32)
        for f in range(od.nfronts - 1, -1, -1):
            lv[f] = 0 if od.parent[f] < 0 else lv[od.parent[f]] + 1
        assert np.array_equal(s["level"], lv)
    finally:
        bfmf.bfmf_destroy(h)


def test_cpp_analysis_matches_oracle_yee():
    n = 6
    rp, ci, v, meta = yee_curlcurl(n, 0.03)
    h = bfmf.bfmf_create(-1)
    try:
        bfmf.bfmf_analyze(h, rp, ci, v, kind=bfmf.BFMF_ORD_YEE, dims=(n, 0, 0), coords=meta["coords"],
                          leaf_max=40, sep_leaf=16)
        od = nd.nd_yee(n, meta["coords"], leaf_max=40, sep_leaf=16)
        _compare(h, od, symbolic(rp, ci, od))
    finally:
        bfmf.bfmf_destroy(h)


def test_error_paths_on_host_handle():
    rp, ci, v, _ = helmholtz_7pt((4, 4, 4), 0.05)
    h = bfmf.bfmf_create(-1)
    try:
        # solve/factor before analyze
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_factor(h)
        assert e.value.status == bfmf.BFMF_E_STATE
        # dims do not match n
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_analyze(h, rp, ci, v, dims=(4, 4, 5))
        assert e.value.status == bfmf.BFMF_E_INVAL
        # column indices out of order
        ci2 = ci.copy()
        ci2[0], ci2[1] = ci2[1], ci2[0]
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_analyze(h, rp, ci2, v, dims=(4, 4, 4))
        assert e.value.status == bfmf.BFMF_E_INVAL
        # non-finite values
        v2 = v.copy()
        v2[3] = np.nan
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_analyze(h, rp, ci, v2, dims=(4, 4, 4))
        assert e.value.status == bfmf.BFMF_E_INVAL
        # a good analysis, then factor on a host-only handle is a state error
        bfmf.bfmf_analyze(h, rp, ci, v, dims=(4, 4, 4), leaf_max=8)
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_factor(h)
        assert e.value.status == bfmf.BFMF_E_STATE
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_solve(h, np.ones(64))
        assert e.value.status == bfmf.BFMF_E_STATE
        assert bfmf.bfmf_status_str(bfmf.BFMF_E_NOCONV)
    finally:
        bfmf.bfmf_destroy(h)


def test_one_hip_runtime_per_process():
    """Importing the binding (before anything else) maps a single libamdhip64:
    the library binds to the HIP runtime torch brings instead of adding a second."""
    import subprocess
    import sys
    code = ("from paper_2007_00202_amd import bfmf\n"
            "import torch\n"
            "paths = set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)\n"
            "print(len(paths))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_hip_sources_are_built_for_gfx950_without_packed_fp32():
    """Every HIP source is compiled for gfx950 with the packed-FP32 instructions switched off (the
    compiler would otherwise emit them from plain float code), and the build covers every .hip and
    .cpp file under csrc."""
    from paper_2007_00202_amd import build as b
    flags = " ".join(b.FLAGS)
    assert "--offload-arch=gfx950" in flags
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
    srcs = {os.path.relpath(s, b.CSRC) for s in b.sources()}
    on_disk = {os.path.relpath(os.path.join(d, f), b.CSRC) for d, _, fs in os.walk(b.CSRC) for f in fs
               if f.endswith((".hip", ".cpp"))}
    assert srcs == on_disk and any(s.endswith(".hip") for s in srcs)


def _user_arrays(od):
    front_ptr = np.concatenate([np.asarray(od.sbeg, np.int64), [od.n]])
    return np.asarray(od.perm, np.int64), front_ptr, np.asarray(od.parent, np.int32)


@pytest.mark.parametrize("dims,leaf,sl", [((8, 8, 8), 64, 16), ((7, 5, 9), 20, 16), ((12, 12, 12), 100, 16)])
def test_user_ordering_reproduces_the_oracle_structures(dims, leaf, sl):
    """A caller-supplied ordering (here the oracle's nested dissection, passed as perm plus front
    tree) gives the oracle's update sets and extend-add maps; each separator's tree halves its
    index range (the balanced tree of the oracle)."""
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=sl)
    sym = symbolic(rp, ci, od)
    perm, fptr, par = _user_arrays(od)
    h = bfmf.bfmf_create(-1)
    try:
        bfmf.bfmf_analyze(h, rp, ci, v, kind=bfmf.BFMF_ORD_USER, sep_leaf=sl, perm=perm, front_ptr=fptr,
                          front_parent=par)
        s = bfmf.bfmf_get_symbolic(h)
        assert np.array_equal(s["perm"], od.perm)
        assert np.array_equal(s["sbeg"], od.sbeg) and np.array_equal(s["send"], od.send)
        assert np.array_equal(s["parent"], od.parent)
        kids = [list(s["child_list"][s["child_ptr"][f]:s["child_ptr"][f + 1]]) for f in range(od.nfronts)]
        assert kids == [list(c) for c in od.children]
        for f in range(od.nfronts):
            assert np.array_equal(s["iu"][s["iu_ptr"][f]:s["iu_ptr"][f + 1]], sym.Iu[f])
            assert np.array_equal(s["map"][s["iu_ptr"][f]:s["iu_ptr"][f + 1]], sym.maps[f])
            nodes = s["sep_nodes"][s["sep_ptr"][f]:s["sep_ptr"][f + 1]]
            assert nodes.tolist() == nd.balanced_tree(int(od.send[f] - od.sbeg[f]), sl)
    finally:
        bfmf.bfmf_destroy(h)


def test_user_ordering_rejects_malformed_input():
    dims = (8, 8, 8)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=16)
    perm, fptr, par = _user_arrays(od)
    root = od.nfronts - 1
    left, right = od.children[root]

    def bad(**kw):
        a = dict(perm=perm, front_ptr=fptr, front_parent=par)
        a.update(kw)
        h = bfmf.bfmf_create(-1)
        try:
            with pytest.raises(bfmf.BfmfError) as e:
                bfmf.bfmf_analyze(h, rp, ci, v, kind=bfmf.BFMF_ORD_USER, sep_leaf=16, **a)
            assert e.value.status == bfmf.BFMF_E_INVAL
            return bfmf.bfmf_last_error(h)
        finally:
            bfmf.bfmf_destroy(h)

    p2 = perm.copy()
    p2[3] = p2[4]
    assert "permutation" in bad(perm=p2)
    q = par.copy()
    q[0] = -1  # a second root
    assert "postorder" in bad(front_parent=q)
    q = par.copy()
    q[left] = 0  # parent before its child
    assert "postorder" in bad(front_parent=q)
    # interleaved subtrees: the first leaf of the left subtree moved under the right child
    first_leaf = 0
    q = par.copy()
    q[first_leaf] = right
    assert "postorder" in bad(front_parent=q)
    f2 = fptr.copy()
    f2[1] = f2[0]  # an empty front
    assert "front_ptr" in bad(front_ptr=f2)
    # separator property: swap one unknown of the first leaf with one of the last leaf of the right
    # subtree, so that both leaves touch the other subtree
    last_leaf = max(f for f in range(od.nfronts) if od.leaf[f])
    p2 = perm.copy()
    i, j = int(od.sbeg[first_leaf]), int(od.sbeg[last_leaf])
    p2[i], p2[j] = p2[j], p2[i]
    assert "separator property" in bad(perm=p2)
