"""GFA reader (the lean structure of Section "CUDA Kernel for Pangenome Graph
Layout": node lengths plus path steps with orientation) on hand-written
fixtures, its error paths, and round trips from the synthetic generator.

The reader is host code in the library; these tests need no GPU except the
last one, which builds a device graph from a GFA file."""
import os

import numpy as np
import pytest

import paper_2409_00876_amd as P
import synth
from paper_2409_00876_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "gfa_reader_fixture.gfa")
R = synth.REV_BIT


def test_fixture_every_record_type():
    """S lines with a sequence, with '*' and LN, and with both; P and W lines
    with reverse steps, revisits on both strands, empty paths, a path that
    names a segment before its S line; L/C/J lines, comments, a CRLF line."""
    g = P.read_gfa(FIXTURE)
    assert g.node_len.tolist() == [7, 3, 2]                   # S-line order: 7, beta, 12
    assert [g.node_name(k) for k in range(3)] == ["7", "beta", "12"]
    assert g.path_names == ["early", "revisit", "empty", "HG002#1#chr6:100-112", "HG002#2#chr6"]
    assert g.path_off.tolist() == [0, 2, 7, 7, 10, 10]
    assert g.step_node.tolist() == [1, 0 | R,                  # early: beta+, 7-
                                    0, 1 | R, 2, 0 | R, 0,     # revisit: 7+, beta-, 12+, 7-, 7+
                                    2, 0 | R, 1]               # walk >12 <7 >beta
    assert g.n_links == 2


def test_parse_equals_read():
    with open(FIXTURE, "rb") as f:
        text = f.read()
    a, b = P.read_gfa(FIXTURE), P.parse_gfa(text)
    for k in ("node_len", "path_off", "step_node"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.path_names == b.path_names
    # no trailing newline, no header
    c = P.parse_gfa(b"S\t1\tA\nP\tp\t1+,1-\t*")
    assert c.node_len.tolist() == [1] and c.step_node.tolist() == [0, R]


def test_empty_text():
    g = P.parse_gfa(b"")
    assert g.n_nodes == 0 and g.n_paths == 0 and g.path_off.tolist() == [0]


@pytest.mark.parametrize("text,status,needle", [
    ("S\t1\tACGT\nS\t1\tAC\n", _lib.ERR_INVALID_ARG, "defined twice"),
    ("S\t1\t*\n", _lib.ERR_INVALID_ARG, "no LN tag"),
    ("S\t1\tACGT\tLN:i:5\n", _lib.ERR_INVALID_ARG, "disagrees"),
    ("S\t1\t*\tLN:i:0\n", _lib.ERR_INVALID_ARG, "length 0"),
    ("S\t1\t*\tLN:i:x\n", _lib.ERR_INVALID_ARG, "bad LN"),
    ("S\t1\t*\tLN:i:4294967296\n", _lib.ERR_RANGE, "2^32"),
    ("S\t1\n", _lib.ERR_INVALID_ARG, "S line"),
    ("S\t1\tA\nP\tp\t1+,2+\t*\n", _lib.ERR_INVALID_ARG, "no S line"),
    ("S\t1\tA\nP\tp\t1\t*\n", _lib.ERR_INVALID_ARG, "orientation"),
    ("S\t1\tA\nP\tp\t1+,,1+\t*\n", _lib.ERR_INVALID_ARG, "empty step"),
    ("S\t1\tA\nP\tp\t1+\t*\nP\tp\t1-\t*\n", _lib.ERR_INVALID_ARG, "used twice"),
    ("S\t1\tA\nP\tp\n", _lib.ERR_INVALID_ARG, "P line"),
    ("S\t1\tA\nW\ts\t0\tc\t*\t*\t1>\n", _lib.ERR_INVALID_ARG, "must start"),
    ("S\t1\tA\nW\ts\t0\tc\t*\t*\t>1<\n", _lib.ERR_INVALID_ARG, "empty segment name"),
    ("S\t1\tA\nW\ts\t0\tc\t*\n", _lib.ERR_INVALID_ARG, "6 fields"),
    ("H\tVN:Z:2.0\n", _lib.ERR_UNSUPPORTED, "GFA 2"),
    ("Sx\t1\tA\n", _lib.ERR_INVALID_ARG, "one letter"),
])
def test_errors(text, status, needle):
    with pytest.raises(P.PgsgdError) as e:
        P.parse_gfa(text)
    assert e.value.status == status
    assert needle in str(e.value)


def test_error_names_the_line():
    with pytest.raises(P.PgsgdError) as e:
        P.parse_gfa("H\tVN:Z:1.0\n# c\nS\t1\tA\nS\t1\tA\n")
    assert "line 4" in str(e.value)


def test_missing_file(tmp_path):
    with pytest.raises(P.PgsgdError) as e:
        P.read_gfa(str(tmp_path / "absent.gfa"))
    assert e.value.status == _lib.ERR_INVALID_ARG and "cannot open" in str(e.value)


def _same(sg, gg):
    assert np.array_equal(gg.node_len, sg.node_len)
    assert np.array_equal(gg.path_off, sg.path_off.astype(np.uint64))
    assert np.array_equal(gg.step_node, sg.step_node)


@pytest.mark.parametrize("walks,names,sequence", [(False, "numeric", False), (True, "numeric", False),
                                                   (False, "text", True), (True, "text", False)])
def test_round_trip_tiny(tmp_path, tiny_synth, walks, names, sequence):
    """synth -> GFA -> reader reproduces node_len, path_offsets and step_node exactly."""
    f = str(tmp_path / "tiny.gfa")
    synth.write_gfa(tiny_synth, f, walks=walks, names=names, sequence=sequence)
    gg = P.read_gfa(f)
    _same(tiny_synth, gg)
    assert gg.path_names[3] == ("hap3#0#chr" if walks else "hap3")
    assert gg.node_name(5) == ("6" if names == "numeric" else "s5")


def test_round_trip_chromosome_model(tmp_path):
    """The chromosome model (lengths 1+Geometric(0.05), 90 paths, inversions
    and SNP alternatives) on a 20,000-node backbone: 1.8M steps."""
    sg = synth.generate(20_000, 0.05, 90, 3)
    assert sg.stats["reverse_visits"] > 0 and sg.stats["alt_nodes"] > 0
    f = str(tmp_path / "chr.gfa")
    synth.write_gfa(sg, f)
    _same(sg, P.read_gfa(f))


def test_sparse_and_mixed_names():
    """Numbers far apart (hash map) and close together (direct table), text
    names, and a number first seen sparse then again: one node per name."""
    text = ("S\t4000000000\tA\nS\t1\tAC\nS\t0\tACG\nS\t007\tACGT\nS\t900000000\tACGTA\nS\tx9\tACGTAC\n"
            "P\tp\t4000000000+,1-,0+,007-,900000000+,x9-,4000000000-,900000000-\t*\n")
    g = P.parse_gfa(text)
    assert g.node_len.tolist() == [1, 2, 3, 4, 5, 6]
    assert g.step_node.tolist() == [0, 1 | R, 2, 3 | R, 4, 5 | R, 0 | R, 4 | R]


def test_property_random_graphs(tmp_path):
    """Random graphs (any node order in the paths, empty paths, revisits):
    write -> read is the identity."""
    hypothesis = pytest.importorskip("hypothesis")
    st = hypothesis.strategies

    @hypothesis.settings(max_examples=60, deadline=None)
    @hypothesis.given(st.data())
    def check(data):
        n = data.draw(st.integers(1, 30))
        lens = data.draw(st.lists(st.integers(1, 50), min_size=n, max_size=n))
        n_paths = data.draw(st.integers(1, 6))
        paths = [data.draw(st.lists(st.tuples(st.integers(0, n - 1), st.booleans()), max_size=25))
                 for _ in range(n_paths)]
        steps = [v | (R if r else 0) for p in paths for v, r in p]
        off = np.cumsum([0] + [len(p) for p in paths]).astype(np.uint64)
        sg = synth.SynthGraph(np.array(lens, np.uint32), off, np.array(steps, np.uint32))
        walks = data.draw(st.booleans())
        names = data.draw(st.sampled_from(["numeric", "text"]))
        f = str(tmp_path / "h.gfa")
        synth.write_gfa(sg, f, walks=walks, names=names)
        _same(sg, P.read_gfa(f))

    check()


@pytest.mark.gpu
def test_graph_from_gfa_samples_the_same_terms(tmp_path, tiny_synth):
    """A device graph built from the GFA text of the tiny graph equals the one
    built from its arrays: same sizes and the same sampled terms."""
    import torch
    f = str(tmp_path / "tiny.gfa")
    synth.write_gfa(tiny_synth, f, walks=True, names="text")
    a = P.Graph.from_synth(tiny_synth)
    b = P.Graph.from_gfa(f)
    assert (a.n_nodes, a.n_paths, a.n_steps, a.d_max) == (b.n_nodes, b.n_paths, b.n_steps, b.d_max)
    for it in (0, 20):
        ta = P.sample_terms(a, it, 0, 8192)
        tb = P.sample_terms(b, it, 0, 8192)
        for x, y in zip(ta, tb):
            assert torch.equal(x, y)
