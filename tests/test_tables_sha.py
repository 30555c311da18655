"""Bit-exact host tables against the oracle at the benchmark's scale: the
subgraph / forest / term lists and the Deg and W tables of eq. (1) of every
graph at 1..4 loops and of the 73 graphs of class (5,0,0), compared through
the SHA-256 digests that tests/golden/make_tables_sha.py wrote from the
oracle."""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_1905_08007_amd as P

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "tables_sha256.json")))


@pytest.mark.parametrize("name", sorted(GOLD))
def test_tables_match_oracle_digests(name):
    rec = GOLD[name]
    cls = rec["class"] or (-1, -1, -1)
    gs = P.enumerate_graphs(rec["loops"], *cls)
    assert len(gs) == rec["ngraphs"]
    s = P.build_forests(gs)
    assert hashlib.sha256(np.ascontiguousarray(s.serialize(), dtype="<i4").tobytes()).hexdigest() == rec["forests"]
    p = P.pdf_create(s)
    h = lambda a: hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()
    for i in range(len(gs)):
        D, W = p.tables(i)
        assert h(D) == rec["deg"][i], (name, i)
        assert h(W) == rec["w"][i], (name, i)
