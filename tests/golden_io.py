"""Reader for the hand-worked fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF = 0x7FFFFFFF


def load_sp_fixture(name):
    """Returns (num_vertices, edges [(s,d,w)], {("sssp"|"bfs", src): int32 vector})."""
    nv, edges, expect = None, [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "vertices":
                nv = int(tok[1])
            elif tok[0] == "edge":
                edges.append(tuple(int(t) for t in tok[1:4]))
            elif tok[0] in ("sssp", "bfs"):
                src = int(tok[1])
                vals = [INF if t == "INF" else int(t) for t in tok[3:]]
                expect[(tok[0], src)] = np.array(vals, np.int32)
    return nv, edges, expect
