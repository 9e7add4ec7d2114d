"""Parser for tests/golden/hand_derived.txt (see the comments in that file)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _floats(line):
    return [float(v) for v in line.split()] if line.strip() else []


def hand_derived_cases():
    lines = []
    with open(os.path.join(GOLDEN, "hand_derived.txt")) as f:
        for raw in f:
            if raw.startswith("#"):
                continue
            lines.append(raw.rstrip("\n"))
    cases, i = [], 0
    while i < len(lines):
        if not lines[i].startswith("case"):
            i += 1
            continue
        name = lines[i].split()[1]
        n, L = (int(v) for v in lines[i + 1].split())
        x = np.array(_floats(lines[i + 2]))
        theta = np.array(_floats(lines[i + 3])).reshape(L, n)
        phi = np.array(_floats(lines[i + 4])).reshape(L, n)
        i += 5
        pairs, expect = [], []
        while lines[i] != "end":
            tok = lines[i].split()
            if tok[0] == "pair":
                pairs.append((int(tok[1]), int(tok[2])))
                expect.append(np.zeros(15))
            else:
                expect[-1][int(tok[0])] = float(tok[1])
            i += 1
        cases.append(dict(name=name, n=n, L=L, x=x, theta=theta, phi=phi,
                          pairs=np.array(pairs, dtype=np.int32), expect=np.stack(expect)))
        i += 1
    return cases
