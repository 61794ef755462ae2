"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def hand_cases():
    """Parse hand_cases.txt into {name: {key: value}}."""
    cases, cur = {}, None
    with open(os.path.join(GOLDEN, "hand_cases.txt")) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest.strip(), "edges": []}
                cases[cur["name"]] = cur
            elif key == "end":
                n = cur["n"]
                for k in ("x0", "jacobi", "gauss_seidel", "exact"):
                    if k in cur:
                        cur[k] = np.array(cur[k], dtype=np.float64).reshape(n, 2)
                cur = None
            elif key == "n":
                cur["n"] = int(rest)
            elif key == "edge":
                a, b = rest.split()
                cur["edges"].append((int(a), int(b)))
            else:
                vals = [float(v) for v in rest.split()]
                cur[key] = vals if len(vals) > 1 or key in ("W",) else vals[0]
    return cases


def ppi_fig4a():
    """(n, edges (m x 2, 0-based), printed coordinates (n x 2)) of Fig. 4(a)."""
    n = None
    coords, edges = {}, []
    with open(os.path.join(GOLDEN, "ppi_fig4a.txt")) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0] == "n":
                n = int(parts[1])
            elif parts[0] == "v":
                coords[int(parts[1])] = (float(parts[2]), float(parts[3]))
            elif parts[0] == "e":
                edges.append((int(parts[1]), int(parts[2])))
    X = np.array([coords[i] for i in range(n)], dtype=np.float64)
    return n, np.array(edges, dtype=np.int64), X
