"""Reader for tests/golden/paper_examples.txt (the paper's printed worked examples)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_examples.txt")


def parse_steps(text: str):
    tg, cm = [], []
    for tok in text.split():
        t, c = tok.split(":")
        tg.append(int(t))
        cm.append(int(c, 0))
    return np.array(tg, dtype=np.uint32), np.array(cm, dtype=np.uint64)


def load_examples(path: str = GOLDEN):
    blocks, cur = {}, None
    with open(path) as f:
        for raw in f:
            line = raw.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                blocks[cur] = {}
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            blocks[cur][k] = v
    out = {}
    for name, b in blocks.items():
        ex = {"name": name, "cite": b["cite"], "M": int(b["M"])}
        ex["target"], ex["cmask"] = parse_steps(b.get("steps", ""))
        if "matrix" in b:
            ex["matrix"] = np.array([[int(x) for x in row.split()] for row in b["matrix"].split("/")],
                                    dtype=np.int64)
        if "expect_sign" in b:
            ex["expect_sign"] = np.array([1.0 if s == "+" else -1.0 for s in b["expect_sign"].split()])
        if "expect_src" in b:
            ex["expect_src"] = np.array([int(x) for x in b["expect_src"].split()], dtype=np.uint64)
        if "rowmap_1based_prefix" in b:
            ex["rowmap_1based_prefix"] = [int(x) for x in b["rowmap_1based_prefix"].split()]
        if "pairs" in b:
            ex["pairs"] = sorted(tuple(int(y) for y in p.split(",")) for p in b["pairs"].split())
        ex["input"] = b.get("input")
        out[name] = ex
    return out
