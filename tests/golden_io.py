"""Reader for the text fixtures under tests/golden/.

A fixture holds ``edge <left> <right> <sign>`` records (sign 1 = positive,
0 = negative, the paper's convention), ``expect ...`` lines and optional
``graph <name> <class>`` headers that start a new graph.  Left and right
labels are numbered per side in order of first appearance.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@dataclass
class Fixture:
    name: str = ""
    label: str = ""
    left: dict = field(default_factory=dict)
    right: dict = field(default_factory=dict)
    edges: list = field(default_factory=list)  # (left index, right index, +1/-1)
    expect: list = field(default_factory=list)

    @property
    def n_u(self):
        return len(self.left)

    @property
    def n_v(self):
        return len(self.right)

    def arrays(self):
        u = np.array([e[0] for e in self.edges], np.int32)
        v = np.array([e[1] for e in self.edges], np.int32)
        s = np.array([e[2] for e in self.edges], np.int8)
        return self.n_u, self.n_v, u, v, s

    def vertex(self, tag):
        """'L<label>' or 'R<label>' -> global index (U first, then V)."""
        side, lab = tag[0], tag[1:]
        return self.left[lab] if side == "L" else self.n_u + self.right[lab]


def load(fname):
    graphs = []
    cur = Fixture(name=fname)
    with open(os.path.join(GOLDEN, fname)) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "graph":
                if cur.edges:
                    graphs.append(cur)
                cur = Fixture(name=tok[1], label=tok[2] if len(tok) > 2 else "")
            elif tok[0] == "edge":
                a = cur.left.setdefault(tok[1], len(cur.left))
                b = cur.right.setdefault(tok[2], len(cur.right))
                cur.edges.append((a, b, 1 if tok[3] == "1" else -1))
            elif tok[0] == "expect":
                cur.expect.append(tok[1:])
            else:
                raise ValueError(f"{fname}: bad line {raw!r}")
    if cur.edges:
        graphs.append(cur)
    return graphs
