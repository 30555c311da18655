"""Oracle pins: graph enumeration against the paper's counts (Table 1)."""
from collections import Counter

from oracle import graphs as GR


def test_table1_class_counts_5loop():
    # Table 1, column N_diag, and "all 3213 integrands" (section "Preliminary
    # numerical results"); orientation-reversed diagrams count once.
    gs = GR.enumerate_graphs(5)
    assert len(gs) == 3213
    c = Counter(g["cls"] for g in gs)
    table1 = {(1, 4, 0): 706, (2, 3, 0): 706, (1, 3, 1): 148, (3, 2, 0): 558,
              (2, 2, 1): 370, (4, 1, 0): 336, (1, 2, 2): 55, (3, 1, 1): 261,
              (5, 0, 0): 73}
    assert dict(c) == table1


def test_low_orders():
    # 1 loop: the Schwinger vertex; 2 loops: 6 raw graphs without lepton loops
    # (ladder, crossed ladder, two corner vertex corrections, two internal
    # self-energies) -> 4 representatives.
    assert len(GR.enumerate_raw(1)) == 1
    assert len(GR.enumerate_raw(2)) == 6
    gs = GR.enumerate_graphs(2)
    assert sorted(g["mult"] for g in gs) == [1, 1, 2, 2]
    assert [len(GR.enumerate_graphs(n)) for n in (3, 4)] == [28, 269]


def test_subgraph_kinds_2loop():
    kinds = []
    for g in GR.enumerate_graphs(2):
        kinds.append(tuple((s["kind"], s["has_x"]) for s in GR.subgraphs(g)))
    # one self-energy, one vertex containing the external vertex (ladder), one
    # vertex not containing it (corner), one graph without subgraphs (crossed)
    assert sorted(kinds) == sorted([(("V", False),), (("S", False),), (("V", True),), ()])


def test_forests_are_nested_or_disjoint():
    for g in GR.enumerate_graphs(4)[:60]:
        subs = GR.subgraphs(g)
        for mask in GR.forests(g):
            idx = [i for i in range(len(subs)) if mask >> i & 1]
            for i in idx:
                for j in idx:
                    if i < j:
                        a, b = subs[i], subs[j]
                        nested = (a["lo"] <= b["lo"] and b["hi"] <= a["hi"]) or (b["lo"] <= a["lo"] and a["hi"] <= b["hi"])
                        assert nested or a["hi"] < b["lo"] or b["hi"] < a["lo"]
