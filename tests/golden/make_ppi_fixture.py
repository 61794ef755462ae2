"""Write ``ppi_fig4a.txt`` from the paper's Fig. 4(a) drawing source.

Fig. 4(a) of the paper draws a 179-vertex protein-protein interaction module
laid out by the SOR method (Sec. 5.4).  Its TikZ source lists every vertex
coordinate and every edge.  This script reads that source from a text file
holding the paper's LaTeX (the figure's TikZ code) and writes the vertex
coordinates and the edge list, 0-based, as a plain-text fixture.  It runs once
when the fixture is (re)made; no test reads the paper.

usage: python tests/golden/make_ppi_fixture.py PAPER_LATEX_FILE
"""
import os
import re
import sys


def parse(text: str):
    start = text.index("(a) PPI network")
    # the first tikzpicture of the figure that ends with the "(a) PPI network" label
    fig = text.rfind("\\begin{figure}", 0, start)
    body = text[fig:start]
    pic_end = body.index("\\end{tikzpicture}")
    pic = body[:pic_end]
    coords = {}
    for m in re.finditer(r"\(\s*([-\d.]+)\s*,\s*([-\d.]+)\s*\)\s*coordinate\s*\((\d+)\)", pic):
        coords[int(m.group(3))] = (m.group(1), m.group(2))
    edges = []
    path = pic[pic.index("\\path\n"):] if "\\path\n" in pic else pic
    for line in path.splitlines():
        line = line.strip()
        m = re.match(r"\((\d+)\)((?:\s*edge\s*\(\d+\))+)", line)
        if not m:
            continue
        a = int(m.group(1))
        for b in re.findall(r"edge\s*\((\d+)\)", m.group(2)):
            edges.append((a, int(b)))
    return coords, edges


def main():
    if len(sys.argv) != 2:
        sys.exit("usage: make_ppi_fixture.py PAPER_LATEX_FILE (the text holding the TikZ source of Fig. 4(a))")
    src = sys.argv[1]
    with open(src, encoding="utf-8", errors="replace") as f:
        text = f.read()
    coords, edges = parse(text)
    n = max(coords)
    assert sorted(coords) == list(range(1, n + 1)), "vertex ids are not 1..n"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ppi_fig4a.txt")
    with open(out, "w") as f:
        f.write("# PPI module of Fig. 4(a) (Sec. 5.4): the SOR layout drawn in the paper.\n")
        f.write("# Parsed from the figure's TikZ source by make_ppi_fixture.py.\n")
        f.write("# Vertices renumbered 0-based (paper id - 1); coordinates in the figure's units.\n")
        f.write("n %d\n" % n)
        f.write("m %d\n" % len(edges))
        for i in range(1, n + 1):
            f.write("v %d %s %s\n" % (i - 1, coords[i][0], coords[i][1]))
        for a, b in edges:
            f.write("e %d %d\n" % (a - 1, b - 1))
    print("wrote", out, "n =", n, "edges =", len(edges))


if __name__ == "__main__":
    main()
