"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects bad host-side arguments with the
documented status before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1606_06508_amd import fh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fh.h", "nrm.h")]


def _declared():
    names = set()
    for header in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:fh|nrm)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_five_entry_points():
    names = _declared()
    for required in ("fh_weights", "fh_eval", "fh_lebesgue", "fh_eval_batched", "fh_eval_backward"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = fh.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings():
    for code in range(10):
        s = fh.status_string(code)
        assert s and s != "unknown status"
    assert fh.status_string(99) == "unknown status"


def lib_pairs_bad_id():
    lib = fh.load()
    assert lib.fh_variant_node_pairs(7, 0) == -1
    return lib.fh_variant_node_pairs(0, 99)


def test_workspace_sizes():
    lib = fh.load()
    assert lib.fh_workspace_size(fh.FH_OP_WEIGHTS, 10, 0, 2, 0) == 256
    a = lib.fh_workspace_size(fh.FH_OP_EVAL, 1001, 10 ** 6, 3, 0)
    a0 = lib.fh_workspace_size(fh.FH_OP_EVAL, 1001, 0, 3, 0)
    b = lib.fh_workspace_size(fh.FH_OP_EVAL, 4097, 10 ** 6, 3, 1)
    # binary64: room for the octet variants' sorted points (16 B each: the
    # point, its node block, its original position); split: the tables only
    assert a - a0 >= 16 * 10 ** 6 and 256 < a0 < b
    assert a % 256 == 0 and b == lib.fh_workspace_size(fh.FH_OP_EVAL, 4097, 0, 3, 1)
    # the adjoint holds a 40-byte binary64 record per point, and the split
    # adjoint a 16-byte binary32 record besides
    bw64 = lib.fh_workspace_size(fh.FH_OP_BACKWARD, 2049, 10 ** 6, 4, 0)
    bw32 = lib.fh_workspace_size(fh.FH_OP_BACKWARD, 2049, 10 ** 6, 4, 1)
    assert bw64 > 40 * 10 ** 6 and bw32 > 56 * 10 ** 6
    # the saved-state adjoint adds four per-point arrays and the point-side
    # sums of up to 64 node tile groups (binary64); split: as the adjoint
    sv64 = lib.fh_workspace_size(fh.FH_OP_BACKWARD_SAVED, 2049, 10 ** 6, 4, 0)
    sv32 = lib.fh_workspace_size(fh.FH_OP_BACKWARD_SAVED, 2049, 10 ** 6, 4, 1)
    assert bw64 + 32 * 10 ** 6 < sv64 <= bw64 + (32 + 8 * 64) * 10 ** 6 + (1 << 30)
    assert bw32 + 48 * 10 ** 6 <= sv32 <= bw32 + 48 * (10 ** 6 + 8192) + (1 << 20)
    big = lib.fh_workspace_size(fh.FH_OP_BACKWARD_SAVED, 10 ** 5, 10 ** 4, 4, 0)
    assert 0 < big < lib.fh_workspace_size(fh.FH_OP_BACKWARD, 10 ** 5, 10 ** 4, 4, 0) + \
        (32 + 8 * 64) * (10 ** 4 + 4096) + (1 << 30)
    # invalid problems report 0
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, 0, 10, 0, 0) == 0
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, 5, 10, 5, 0) == 0
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, 5, -1, 1, 0) == 0
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, 5, 10, 1, 7) == 0


# Fake, never-dereferenced device addresses: every call below must return
# before any kernel launch or HIP call.
P = ctypes.c_void_p(0x100000)
P2 = ctypes.c_void_p(0x200000)


@pytest.mark.parametrize("args,code", [
    (dict(nodes=None), fh.FH_E_ARG),
    (dict(n=0), fh.FH_E_ARG),
    (dict(d=-1), fh.FH_E_DEGREE),
    (dict(d=10), fh.FH_E_DEGREE),
    (dict(m=-1), fh.FH_E_ARG),
    (dict(x=None), fh.FH_E_ARG),
    (dict(r=None), fh.FH_E_ARG),
    (dict(values=None), fh.FH_E_ARG),
    (dict(prec=5), fh.FH_E_ARG),
    (dict(ws=None), fh.FH_E_WORKSPACE),
    (dict(ws_bytes=100), fh.FH_E_WORKSPACE),
    (dict(ws=ctypes.c_void_p(0x100008)), fh.FH_E_WORKSPACE),
])
def test_eval_host_validation(args, code):
    lib = fh.load()
    a = dict(nodes=P, values=P, n=10, d=3, x=P, m=100, r=P2, lam=None, w=None, prec=0, ws=P,
             ws_bytes=1 << 30, stream=None)
    a.update(args)
    got = lib.fh_eval(a["nodes"], a["values"], a["n"], a["d"], a["x"], a["m"], a["r"], a["lam"],
                      a["w"], a["prec"], a["ws"], a["ws_bytes"], a["stream"])
    assert got == code


def test_saved_adjoint_host_validation():
    """fh_eval_forward / fh_eval_backward_saved reject bad host arguments
    before any launch."""
    lib = fh.load()
    ws = 1 << 40
    fwd = lambda **k: lib.fh_eval_forward(*[k.get(a, b) for a, b in (
        ("nodes", P), ("values", P), ("n", 10), ("d", 3), ("x", P), ("m", 100), ("r", P2),
        ("dr", None), ("prec", 0), ("ws", P), ("ws_bytes", ws), ("stream", None))])
    bwd = lambda **k: lib.fh_eval_backward_saved(*[k.get(a, b) for a, b in (
        ("nodes", P), ("n", 10), ("d", 3), ("x", P), ("m", 100), ("dr", None), ("g", P2),
        ("gv", P2), ("gx", P2), ("gn", P2), ("prec", 0), ("ws", P), ("ws_bytes", ws),
        ("stream", None))])
    for call in (fwd, bwd):
        assert call(nodes=None) == fh.FH_E_ARG
        assert call(d=10) == fh.FH_E_DEGREE
        assert call(m=-1) == fh.FH_E_ARG
        assert call(x=None) == fh.FH_E_ARG
        assert call(prec=3) == fh.FH_E_ARG
        assert call(ws=None) == fh.FH_E_WORKSPACE
        assert call(ws_bytes=4096) == fh.FH_E_WORKSPACE
        assert call(ws=ctypes.c_void_p(0x100008)) == fh.FH_E_WORKSPACE
    assert fwd(values=None) == fh.FH_E_ARG
    assert fwd(r=None) == fh.FH_E_ARG
    assert bwd(g=None) == fh.FH_E_ARG
    # the forward's size is the one checked
    need = lib.fh_workspace_size(fh.FH_OP_BACKWARD_SAVED, 10, 100, 3, 0)
    assert need > lib.fh_workspace_size(fh.FH_OP_BACKWARD, 10, 100, 3, 0)
    assert fwd(ws_bytes=need - 1) == fh.FH_E_WORKSPACE
    assert bwd(ws_bytes=need - 1) == fh.FH_E_WORKSPACE


def test_weights_and_lebesgue_host_validation():
    lib = fh.load()
    assert lib.fh_weights(P, 5, 5, P2, P, 256, None) == fh.FH_E_DEGREE
    assert lib.fh_weights(P, 5, 1, None, P, 256, None) == fh.FH_E_ARG
    assert lib.fh_weights(P, 5, 1, P2, None, 256, None) == fh.FH_E_WORKSPACE
    assert lib.fh_lebesgue(P, 5, 1, P, 10, None, None, 0, P, 1 << 20, None) == fh.FH_E_ARG
    assert lib.fh_lebesgue(P, 5, 7, P, 10, P2, None, 0, P, 1 << 20, None) == fh.FH_E_DEGREE


def test_lebesgue_max_host_validation_and_workspace():
    lib = fh.load()
    a = lib.fh_workspace_size(fh.FH_OP_EVAL, 1001, 0, 3, 1)  # the node tables
    b = lib.fh_workspace_size(fh.FH_OP_LEBESGUE_MAX, 1001, 0, 3, 0)
    assert b >= a + 2 * 8 * 1000 and b % 256 == 0
    assert lib.fh_workspace_size(fh.FH_OP_LEBESGUE_MAX, 1, 0, 0, 0) > 0

    def call(**kw):
        a = dict(nodes=P, n=10, d=3, w=None, samples=256, rounds=5, lam=P2, loc=None, best=None,
                 prec=0, ws=P, ws_bytes=1 << 30)
        a.update(kw)
        return lib.fh_lebesgue_max(a["nodes"], a["n"], a["d"], a["w"], a["samples"], a["rounds"],
                                   a["lam"], a["loc"], a["best"], a["prec"], a["ws"],
                                   a["ws_bytes"], None)

    assert call(nodes=None) == fh.FH_E_ARG
    assert call(d=10) == fh.FH_E_DEGREE
    for bad in (dict(samples=0), dict(samples=513), dict(rounds=0), dict(rounds=65),
                dict(lam=None), dict(prec=4)):
        assert call(**bad) == fh.FH_E_ARG, bad
    assert call(prec=1) == fh.FH_E_UNSUPPORTED
    assert call(ws=None) == fh.FH_E_WORKSPACE
    assert call(ws_bytes=300) == fh.FH_E_WORKSPACE


def test_variant_tables_and_tuner_api():
    """The tuner interface: enumerate variants, record / override / release
    a choice, and reject bad arguments -- all host-side."""
    for prec in ("fp64", "split"):
        vs = fh.variants(prec)
        assert len(vs) >= 4
        assert len({v[0] for v in vs}) == len(vs)
        for vid, p, g, s in vs:
            assert p in (1, 2, 4, 8) and g in (1, 4, 8) and s in (1, 2, 4)
        base = fh.tune_get(prec, 777, 123456)
        assert 0 <= base < len(vs)
        other = (base + 1) % len(vs)
        fh.tune_set(prec, 777, 123456, other)
        assert fh.tune_get(prec, 777, 123456) == other
        assert fh.tune_get(prec, 777, 10 ** 8) != -1          # other bucket untouched
        fh.tune_force(prec, base)
        assert fh.tune_get(prec, 777, 123456) == base          # force wins
        fh.tune_force(prec, -1)
        fh.tune_set(prec, 777, 123456, -1)                      # remove entry
        assert fh.tune_get(prec, 777, 123456) == base
    lib = fh.load()
    assert lib.fh_tune_force(0, 999) == fh.FH_E_ARG
    assert lib.fh_tune_set(0, 0, 10, 1) == fh.FH_E_ARG
    assert lib.fh_tune_set(5, 10, 10, 1) == fh.FH_E_ARG
    assert lib.fh_variant_count(7) == 0


def test_batched_variant_tables():
    """Batched variants: binary64 over points per lane, node split, Lebesgue
    block and passes per strip; split over points per lane and passes.  The
    strip (points of one work item) is 64 P (4 / S) Q, split 256 P Q; the
    first three binary64 variants are the plain single-pass shapes with
    P = 1, 2, 4."""
    f64 = fh.variants("batched_fp64")
    assert len(f64) >= 12 and [v[1:] for v in f64[:3]] == [(1, 8, 1), (2, 8, 1), (4, 8, 1)]
    strips = set()
    for vid, p, g, s in f64:
        st = fh.variant_strip_points("batched_fp64", vid)
        assert st % (64 * p * (4 // s)) == 0 and st // (64 * p * (4 // s)) in (1, 4)
        strips.add(st)
        assert fh.variant_lebesgue_block("batched_fp64", vid) in (0, 16)
    assert len(strips) >= 4
    sp = fh.variants("batched_split")
    assert len(sp) >= 6
    for vid, p, g, s in sp:
        assert g == 4 and s == 1
        st = fh.variant_strip_points("batched_split", vid)
        assert st % (256 * p) == 0 and st // (256 * p) in (1, 4)
    assert fh.variant_strip_points("fp64", 16) == 64 * 2 * 1   # P = 2, S = 4
    assert fh.variant_strip_points("split", 9) == 256 * 2
    lib = fh.load()
    assert lib.fh_variant_strip_points(7, 0) == -1 and lib.fh_variant_strip_points(2, 999) == -1
    assert lib.fh_batch_variant(None) == -1 and lib.fh_batch_strip_points(None) == -1


def test_lebesgue_block_variants():
    """Binary64 variants 15..26 take the Lebesgue sum by blocks of 16 nodes,
    19..26 of them summing each block by node pairs and 25..26 the blocks
    far from a point by octets (their shapes are those of pair variants 22
    and 20); split variants 8..11 by
    tiles of 32 (the block counterparts of plain shapes); every other single
    variant uses plain sums.  Batched split variants take tiles of 32,
    batched binary64 ones plain sums."""
    blocks = {vid: fh.variant_lebesgue_block("fp64", vid) for vid, *_ in fh.variants("fp64")}
    assert {vid for vid, u in blocks.items() if u} == set(range(15, 27))
    assert set(blocks.values()) == {0, 16}
    pairs = {vid for vid, *_ in fh.variants("fp64") if fh.variant_node_pairs("fp64", vid)}
    assert pairs == set(range(19, 27))
    octets = {vid for vid, *_ in fh.variants("fp64") if fh.variant_octets("fp64", vid)}
    assert octets == {25, 26}
    assert not any(fh.variant_octets(f, 0) for f in ("split", "batched_fp64", "batched_split"))
    assert not any(fh.variant_node_pairs(f, 0) for f in ("split", "batched_fp64", "batched_split"))
    shapes = {vid: (p, g, s) for vid, p, g, s in fh.variants("fp64")}
    for vid in range(15, 27):
        assert shapes[vid] in [shapes[v] for v, u in blocks.items() if u == 0]
    assert shapes[25] == shapes[22] and shapes[26] == shapes[20]
    assert lib_pairs_bad_id() == -1
    sb = {vid: fh.variant_lebesgue_block("split", vid) for vid, *_ in fh.variants("split")}
    assert {vid for vid, u in sb.items() if u} == {8, 9, 10, 11} and set(sb.values()) == {0, 32}
    sshapes = {vid: (p, g, s) for vid, p, g, s in fh.variants("split")}
    for vid in (8, 9, 10, 11):
        assert sshapes[vid] in [sshapes[v] for v, u in sb.items() if u == 0]
    bb = {vid: fh.variant_lebesgue_block(2, vid) for vid, *_ in fh.variants(2)}
    assert set(bb.values()) == {0, 16}
    for vid, *_ in fh.variants(3):
        assert fh.variant_lebesgue_block(3, vid) == 32
    lib = fh.load()
    assert lib.fh_variant_lebesgue_block(0, 99) == -1
    assert lib.fh_variant_lebesgue_block(7, 0) == -1
    with pytest.raises(fh.FhError):
        fh.variant_lebesgue_block("fp64", -1)


def test_normalize_entry_points_and_host_validation():
    """The six normalization entry points are declared and reject bad
    arguments before any launch."""
    lib = fh.load()
    names = _declared()
    dummy = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation
    for dim in (2, 3, 4):
        for sfx in ("f32", "f64"):
            name = f"nrm_normalize{dim}_{sfx}"
            assert name in names
            fn = getattr(lib, name)
            assert fn(None, 0, None, None, 0, 0, None) == fh.FH_OK          # nothing to do
            assert fn(None, -1, None, None, 0, 0, None) == fh.FH_E_ARG
            assert fn(None, 4, dummy, dummy, 0, 0, None) == fh.FH_E_ARG     # no input
            assert fn(dummy, 4, None, None, 0, 0, None) == fh.FH_E_ARG     # no output
            assert fn(dummy, 4, dummy, dummy, 2, 0, None) == fh.FH_E_ARG   # layout
            assert fn(dummy, 4, dummy, dummy, 0, 4, None) == fh.FH_E_ARG   # method
            pivot = fn(dummy, 4, dummy, dummy, 0, 2, None) if dim != 3 else None
            assert dim == 3 or pivot == fh.FH_E_ARG                         # Algorithm 2 is 3D


def test_multi_host_validation_and_workspace():
    lib = fh.load()
    one = lib.fh_workspace_size(fh.FH_OP_EVAL, 1001, 0, 3, 0)
    assert lib.fh_multi_workspace_size(1001, 9) > one
    assert lib.fh_multi_workspace_size(1001, 0) == 0 and lib.fh_multi_workspace_size(1001, 65) == 0
    assert lib.fh_multi_workspace_size(0, 4) == 0

    def call(K=3, degs=(1, 2, 3), n=10, **kw):
        a = dict(nodes=P, values=P, x=P, m=100, r=P2, lam=None, ws=P, ws_bytes=1 << 30)
        a.update(kw)
        d = (ctypes.c_int32 * max(len(degs), 1))(*degs)
        return lib.fh_eval_multi(a["nodes"], a["values"], n, d, K, a["x"], a["m"], a["r"],
                                 a["lam"], a["ws"], a["ws_bytes"], None)

    assert call(K=0, degs=()) == fh.FH_E_ARG
    assert call(K=65, degs=tuple([1] * 65)) == fh.FH_E_ARG
    assert call(degs=(1, 10, 3)) == fh.FH_E_DEGREE
    assert call(degs=(1, -1, 3)) == fh.FH_E_DEGREE
    assert call(nodes=None) == fh.FH_E_ARG and call(values=None) == fh.FH_E_ARG
    assert call(r=None) == fh.FH_E_ARG and call(m=-1) == fh.FH_E_ARG
    assert call(ws=None) == fh.FH_E_WORKSPACE and call(ws_bytes=512) == fh.FH_E_WORKSPACE


def test_node_count_limit():
    """n above FH_MAX_NODES (node loops index with 32-bit integers) is refused
    on the host by every entry point that takes a node count."""
    lib = fh.load()
    hdr = open(HEADERS[0]).read()
    assert re.search(r"#define FH_MAX_NODES \(1LL << 28\)", hdr) and fh.FH_MAX_NODES == 1 << 28
    big = fh.FH_MAX_NODES + 1
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, fh.FH_MAX_NODES, 10, 3, 0) > 0
    for op in (fh.FH_OP_WEIGHTS, fh.FH_OP_EVAL, fh.FH_OP_BACKWARD, fh.FH_OP_LEBESGUE_MAX):
        assert lib.fh_workspace_size(op, big, 10, 3, 0) == 0, op
    assert lib.fh_multi_workspace_size(big, 2) == 0
    assert lib.fh_weights(P, big, 3, P2, P, 1 << 62, None) == fh.FH_E_ARG
    assert lib.fh_eval(P, P, big, 3, P, 100, P2, None, None, 0, P, 1 << 62, None) == fh.FH_E_ARG
    assert lib.fh_lebesgue(P, big, 3, P, 100, P2, None, 0, P, 1 << 62, None) == fh.FH_E_ARG
    assert lib.fh_eval_prepared(P, 1 << 62, big, 0, P, 100, P2, None, None) == fh.FH_E_ARG
    assert lib.fh_eval_deriv(P, P, big, 3, P, 100, None, P2, None, 0, P, 1 << 62,
                             None) == fh.FH_E_ARG
    assert lib.fh_eval_backward(P, P, big, 3, P, 100, P2, P2, P2, P2, 0, P, 1 << 62,
                                None) == fh.FH_E_ARG
    assert lib.fh_lebesgue_max(P, big, 3, None, 256, 5, P2, None, None, 0, P, 1 << 62,
                               None) == fh.FH_E_ARG
    d = (ctypes.c_int32 * 2)(3, 3)
    assert lib.fh_eval_multi(P, P, big, d, 2, P, 100, P2, None, P, 1 << 62, None) == fh.FH_E_ARG
    h = ctypes.c_void_p()
    n_host = (ctypes.c_int64 * 2)(5, big)
    d_host = (ctypes.c_int32 * 2)(1, 1)
    m_host = (ctypes.c_int64 * 2)(10, 10)
    assert lib.fh_batch_create(ctypes.byref(h), 2, n_host, d_host, m_host, P, P, P, P2, None, 0,
                               None) == fh.FH_E_ARG
    assert h.value is None


def test_noalloc_host_validation_and_limit():
    """fh_eval_noalloc refuses bad arguments, and node counts whose table
    does not fit its fixed device array, before any HIP call; the header's
    limit is the largest node count whose table fits."""
    lib = fh.load()
    hdr = open(HEADERS[0]).read()
    cap = int(re.search(r"#define FH_NOALLOC_SCRATCH_BYTES \(\(size_t\)2 << 20\)", hdr)
              and 2 << 20)
    top = int(re.search(r"#define FH_NOALLOC_MAX_NODES (\d+)LL", hdr).group(1))
    assert top == fh.FH_NOALLOC_MAX_NODES
    # the node tables (a split-precision evaluation workspace holds just
    # those; the array never holds the octet variants' sorted points)
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, top, 10, 3, 1) <= cap
    assert lib.fh_workspace_size(fh.FH_OP_EVAL, top + 1, 10, 3, 1) > cap

    def call(**kw):
        a = dict(nodes=P, values=P, n=10, d=3, x=P, m=100, r=P2, lam=None, w=None, prec=0)
        a.update(kw)
        return lib.fh_eval_noalloc(a["nodes"], a["values"], a["n"], a["d"], a["x"], a["m"],
                                   a["r"], a["lam"], a["w"], a["prec"], None)

    assert call(n=top + 1) == fh.FH_E_TOO_LARGE
    assert call(n=fh.FH_MAX_NODES + 1) == fh.FH_E_ARG
    assert call(nodes=None) == fh.FH_E_ARG and call(values=None) == fh.FH_E_ARG
    assert call(n=0) == fh.FH_E_ARG and call(m=-1) == fh.FH_E_ARG
    assert call(x=None) == fh.FH_E_ARG and call(r=None) == fh.FH_E_ARG
    assert call(d=10) == fh.FH_E_DEGREE and call(d=-1) == fh.FH_E_DEGREE
    assert call(prec=2) == fh.FH_E_ARG
    assert "noalloc" in fh.status_string(fh.FH_E_TOO_LARGE)


def test_prepare_many_host_validation():
    lib = fh.load()
    ws = (ctypes.c_void_p * 3)(0x100000, 0x200000, 0x300000)

    def call(K=3, degs=(1, 2, 3), n=10, prec=0, wss=ws, ws_bytes=1 << 30, nodes=P):
        d = (ctypes.c_int32 * max(len(degs), 1))(*degs)
        return lib.fh_prepare_many(nodes, P, n, d, K, prec, wss, ws_bytes, None)

    assert call(K=0, degs=()) == fh.FH_E_ARG
    assert call(K=17, degs=tuple([1] * 17),
                wss=(ctypes.c_void_p * 17)(*[0x100000 * (i + 1) for i in range(17)])) == fh.FH_E_ARG
    assert call(n=0) == fh.FH_E_ARG and call(nodes=None) == fh.FH_E_ARG
    assert call(prec=1) == fh.FH_E_UNSUPPORTED and call(prec=3) == fh.FH_E_ARG
    assert call(degs=(1, 10, 3)) == fh.FH_E_DEGREE
    assert call(ws_bytes=300) == fh.FH_E_WORKSPACE
    assert call(wss=(ctypes.c_void_p * 3)(0x100000, None, 0x300000)) == fh.FH_E_WORKSPACE
    assert call(wss=(ctypes.c_void_p * 3)(0x100000, 0x200008, 0x300000)) == fh.FH_E_WORKSPACE
    assert call(wss=(ctypes.c_void_p * 3)(0x100000, 0x200000, 0x100000)) == fh.FH_E_ARG
    assert lib.fh_prepare_many(P, P, 10, None, 3, 0, ws, 1 << 30, None) == fh.FH_E_ARG


def test_eval_prepared_many_host_validation():
    """Host-checkable errors of fh_eval_prepared_many return before any
    launch (fake device addresses: none is dereferenced)."""
    lib = fh.load()
    VP = ctypes.c_void_p
    ws = (VP * 3)(0x100000, 0x200000, 0x300000)
    outs = (VP * 3)(0x400000, 0x500000, 0x600000)

    def call(K=3, n=10, prec=0, wss=ws, ws_bytes=1 << 30, x=P, m=100, r=outs, lam=outs):
        return lib.fh_eval_prepared_many(wss, ws_bytes, K, n, prec, x, m, r, lam, None)

    assert call(K=0) == fh.FH_E_ARG
    assert call(K=17, wss=(VP * 17)(*[0x100000 * (i + 1) for i in range(17)]),
                r=None, lam=(VP * 17)(*[0x100000 * (i + 40) for i in range(17)])) == fh.FH_E_ARG
    assert call(n=0) == fh.FH_E_ARG and call(n=fh.FH_MAX_NODES + 1) == fh.FH_E_ARG
    assert call(m=-1) == fh.FH_E_ARG and call(x=None) == fh.FH_E_ARG
    assert call(r=None, lam=None) == fh.FH_E_ARG
    assert call(wss=None) == fh.FH_E_ARG
    assert call(prec=1) == fh.FH_E_UNSUPPORTED and call(prec=3) == fh.FH_E_ARG
    assert call(ws_bytes=300) == fh.FH_E_WORKSPACE
    assert call(wss=(VP * 3)(0x100000, None, 0x300000)) == fh.FH_E_WORKSPACE
    assert call(wss=(VP * 3)(0x100000, 0x200008, 0x300000)) == fh.FH_E_WORKSPACE
    assert call(r=(VP * 3)(0x400000, None, 0x600000)) == fh.FH_E_ARG
    assert call(lam=(VP * 3)(0x400000, 0x500000, None)) == fh.FH_E_ARG
    # m = 0: validated, nothing launched
    assert call(m=0, x=None) == fh.FH_OK


def _run_py(code, env_extra):
    import subprocess
    import sys
    env = dict(os.environ, **env_extra)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                          timeout=120, env=env, cwd=ROOT)


def test_fh_log_reports_choices():
    """FH_LOG=1: every new (shape, variant) choice is reported on stderr with
    its source, once."""
    code = ("from paper_1606_06508_amd import fh\n"
            "fh.tune_get('fp64', 1001, 10**6); fh.tune_get('fp64', 1001, 10**6)\n"
            "fh.tune_get('batched_split', 1041, 204421648)\n")
    p = _run_py(code, {"FH_LOG": "1"})
    assert p.returncode == 0, p.stderr
    lines = [ln for ln in p.stderr.splitlines() if ln.startswith("[fh]")]
    assert lines == ["[fh] fp64 n=1001 m=1000000: variant 25 (built-in)",
                     "[fh] batched_split n=1041 m=204421648: variant 5 (built-in)"], p.stderr
    q = _run_py(code, {"FH_LOG": "0"})
    assert q.returncode == 0 and "[fh]" not in q.stderr


def test_autotune_cache_for_another_architecture_is_ignored(tmp_path):
    """A table saved for another architecture is not installed (and the
    library says so under FH_LOG); a missing file is reported too."""
    import json
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"arch": "gfx000", "entries": [
        {"precision": "fp64", "n": 1001, "m": 1000000, "lambda": 1, "variant": 3,
         "ms": 0.2, "all_ms": {"3": 0.2, "17": 0.3}}]}))
    code = "from paper_1606_06508_amd import fh\nprint(fh.tune_get('fp64', 1001, 10**6))\n"
    p = _run_py(code, {"FH_LOG": "1", "FH_AUTOTUNE_CACHE": str(path)})
    assert p.returncode == 0, p.stderr
    assert p.stdout.strip() == "25"
    assert "made for 'gfx000'" in p.stderr and "ignored" in p.stderr
    q = _run_py(code, {"FH_LOG": "1", "FH_AUTOTUNE_CACHE": str(tmp_path / "missing.json")})
    assert q.stdout.strip() == "25" and "cannot open" in q.stderr
