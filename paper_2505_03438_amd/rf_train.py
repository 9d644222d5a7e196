"""Train the Random Forest selection model and write it out as C++ tables.

Sec. 5.3: a random forest classifier (100 trees) maps the live statistics of
Sec. 4 to the configuration to use; it is trained on scenarios whose
configurations were all trialled.  Here the training data are Full Search
trials on MI355X over generative scenarios (workloads.selection_scenarios,
recorded by ``python -m paper_2505_03438_amd.fullsearch_table --set
selection`` into data/selection_fullsearch.jsonl); training runs offline with
scikit-learn, and the fitted trees are written to csrc/rf_model.h, which the
library's own tree evaluator reads (no Python in the tuning loop).

    python -m paper_2505_03438_amd.rf_train [--data FILE] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "data", "selection_fullsearch.jsonl")
OUT = os.path.join(HERE, "csrc", "rf_model.h")
N_TREES = 100
SEED = 0


def load(path: str = DATA):
    rows = [json.loads(line) for line in open(path) if line.strip()]
    X = np.array([r["features"] for r in rows], dtype=np.float64)
    y = np.array([int(r["label"]) for r in rows], dtype=np.int64)
    return X, y


def fit(X, y):
    from sklearn.ensemble import RandomForestClassifier
    return RandomForestClassifier(n_estimators=N_TREES, random_state=SEED).fit(X, y)


def write_header(model, path: str = OUT, source: str = "data/selection_fullsearch.jsonl"):
    classes = [int(c) for c in model.classes_]
    nodes, proba, roots = [], [], []
    for est in model.estimators_:
        t = est.tree_
        roots.append(len(nodes))
        base = len(nodes)
        for k in range(t.node_count):
            if t.children_left[k] < 0:
                nodes.append((-1, 0.0, -1, -1, len(proba)))
                proba.extend(float(v) for v in t.value[k][0])
            else:
                nodes.append((int(t.feature[k]), float(t.threshold[k]), base + int(t.children_left[k]),
                              base + int(t.children_right[k]), -1))
    out = []
    out.append("// Random Forest selection model (Sec. 5.3): %d trees over the 8 live" % len(model.estimators_))
    out.append("// statistics, written by rf_train.py from %s." % source)
    out.append("// Generated file; regenerate instead of editing.")
    out.append("#pragma once")
    out.append("")
    out.append("#include <stdint.h>")
    out.append("")
    out.append("namespace mdlj {")
    out.append("namespace rf {")
    out.append("")
    out.append("struct Node {")
    out.append("    int32_t feature;   // statistic index, -1 for a leaf")
    out.append("    double threshold;  // go left iff (float) statistic <= threshold")
    out.append("    int32_t left, right;")
    out.append("    int32_t proba;     // leaf: offset of its class fractions")
    out.append("};")
    out.append("")
    out.append("constexpr int kTrees = %d;" % len(roots))
    out.append("constexpr int kClasses = %d;" % len(classes))
    out.append("// class k means tuning-space configuration kConfig[k]")
    out.append("constexpr int kConfig[kClasses] = {%s};" % ", ".join(str(c) for c in classes))
    out.append("constexpr int kRoot[kTrees] = {")
    for i in range(0, len(roots), 12):
        out.append("    " + ", ".join(str(r) for r in roots[i:i + 12]) + ",")
    out.append("};")
    out.append("constexpr Node kNodes[%d] = {" % len(nodes))
    for f, th, l, r, p in nodes:
        out.append("    {%d, %s, %d, %d, %d}," % (f, float(th).hex(), l, r, p))
    out.append("};")
    out.append("constexpr double kProba[%d] = {" % len(proba))
    for i in range(0, len(proba), 4):
        out.append("    " + ", ".join(float(v).hex() for v in proba[i:i + 4]) + ",")
    out.append("};")
    out.append("")
    out.append("}  // namespace rf")
    out.append("}  // namespace mdlj")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--data", default=DATA)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    X, y = load(args.data)
    model = fit(X, y)
    write_header(model, args.out, os.path.relpath(args.data, HERE))
    print("trained on %d scenarios, classes %s, training accuracy %.3f -> %s"
          % (len(y), list(model.classes_), model.score(X, y), args.out))


if __name__ == "__main__":
    main()
