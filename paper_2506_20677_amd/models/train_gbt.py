#!/usr/bin/env python3
"""Fits the strategy selector of Sec. III-H (gradient-boosted trees over the
features (n, k = span + 1, H)) to labels measured on the target GPU by
collect_labels.py, and writes it in the library's text format (the format
ahs_model_load and the oracle's ref_model_load parse).

The class of a workload is its fastest forced strategy (COUNTING, RADIX,
QUICK); each workload is weighted by how much a wrong choice would cost
(log of the slowest feasible time over the fastest).  Training uses
scikit-learn's GradientBoostingClassifier (multinomial deviance); the export
keeps its arithmetic: class score = initial raw score + learning rate x the
leaf values of the class's trees, and the largest score wins.  scikit-learn
sends x <= t to the left child, the library x < t, so thresholds are moved
to the next double above.  The trees are fitted over log2 n, log2 k and H,
so that a split between two measured sizes falls at their geometric mean
(an input halfway between 2^24 and 2^26 keys in log scale follows the
nearer one); the export turns a log threshold t back into 2^t, which leaves
every training row on the same side.  log2 k is rounded up to a multiple of
1/4 first: spans within a factor 2^(1/4) look alike, so the trees cannot
split between the random spans of two draws of one family (say 4.24e9 and
4.27e9), and k = 65,536 (counting feasible) stays apart from 65,537.  A
threshold between two such steps is exported at the step below it, as
k < next double above 2^step.  The written model is then re-evaluated with the
library's own evaluator (ahs_model_predict, a host function), which must
reproduce scikit-learn's class on every training row.
"""
import argparse
import csv
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CLASSES = ("counting", "radix", "quick")


def load(path):
    rows = list(csv.DictReader(open(path)))
    X, y, w, times = [], [], [], []
    for r in rows:
        t = [float(r["t_counting"]), float(r["t_radix"]), float(r["t_quick"])]
        X.append([float(r["n"]), float(r["span"]) + 1.0, float(r["entropy_bits"])])
        y.append(CLASSES.index(r["best"]))
        finite = [v for v in t if math.isfinite(v)]
        w.append(0.1 + math.log(max(finite) / min(finite)))
        times.append(t)
    return rows, np.array(X), np.array(y), np.array(w), np.array(times)


K_STEPS = 4  # log2 k in steps of 1 / K_STEPS


def fit_space(X):
    """Columns the trees are fitted over: log2 n, log2 k rounded up to a
    step, H."""
    Z = np.array(X, dtype=np.float64)
    Z[:, 0] = np.log2(Z[:, 0])
    Z[:, 1] = np.ceil(np.log2(Z[:, 1]) * K_STEPS) / K_STEPS
    return Z


def export(clf, path):
    lr = clf.learning_rate
    base = clf._raw_predict_init(np.zeros((1, 3)))[0]
    lines = ["ahs-gbt 1", "num_class 3", "base_score " + " ".join(repr(float(b)) for b in base)]
    trees = []
    for stage in clf.estimators_:
        for cls, est in enumerate(stage):
            t = est.tree_
            nodes = []
            for i in range(t.node_count):
                if t.children_left[i] == -1:
                    nodes.append(f"{i} leaf {float(t.value[i][0][0]) * lr!r}")
                else:
                    thr = float(t.threshold[i])
                    if int(t.feature[i]) == 1:  # stepped log2 k: the step at or below t
                        thr = float(2.0 ** (math.floor(thr * K_STEPS) / K_STEPS))
                    elif int(t.feature[i]) == 0:  # log2 n
                        thr = float(2.0 ** thr)
                    thr = float(np.nextafter(thr, np.inf))
                    nodes.append(f"{i} split {int(t.feature[i])} {thr!r} {int(t.children_left[i])} "
                                 f"{int(t.children_right[i])}")
            trees.append((cls, nodes))
    lines.append(f"num_trees {len(trees)}")
    for cls, nodes in trees:
        lines.append(f"tree {cls} {len(nodes)}")
        lines.extend(nodes)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def held_out_regret(times, pred):
    """Time of the predicted strategy over the best time, per row (inf if infeasible)."""
    out = []
    for t, c in zip(times, pred):
        out.append(t[c] / np.nanmin(t) if math.isfinite(t[c]) else float("inf"))
    return np.array(out)


def cross_validate(X, y, w, times):
    from sklearn.ensemble import GradientBoostingClassifier
    from sklearn.model_selection import KFold

    X = fit_space(X)
    folds = list(KFold(n_splits=5, shuffle=True, random_state=0).split(X))
    print("stages depth | held-out accuracy | mean time over best | worst")
    for depth in (1, 2, 3):
        for stages in (5, 10, 20, 40):
            acc, reg = [], []
            for tr, te in folds:
                clf = GradientBoostingClassifier(n_estimators=stages, max_depth=depth, learning_rate=0.3,
                                                 random_state=0)
                clf.fit(X[tr], y[tr], sample_weight=w[tr])
                p = clf.predict(X[te])
                acc.append(np.mean(p == y[te]))
                reg.extend(held_out_regret(times[te], p))
            reg = np.array(reg)
            fin = reg[np.isfinite(reg)]
            print(f"{stages:6d} {depth:5d} | {np.mean(acc):.3f} | {np.mean(fin):.4f} | "
                  f"{reg.max():.2f} ({int((~np.isfinite(reg)).sum())} infeasible)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--labels", default=os.path.join(HERE, "mi355x_labels.csv"))
    ap.add_argument("--out", default=os.path.join(HERE, "mi355x_selector.gbt"))
    ap.add_argument("--trees", type=int, default=10)
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--cv", action="store_true",
                    help="only report 5-fold cross-validation over a grid of tree counts and depths")
    args = ap.parse_args()
    from sklearn.ensemble import GradientBoostingClassifier

    rows, X, y, w, times = load(args.labels)
    if args.cv:
        cross_validate(X, y, w, times)
        return
    clf = GradientBoostingClassifier(n_estimators=args.trees, max_depth=args.depth, learning_rate=0.3,
                                     random_state=0)
    clf.fit(fit_space(X), y, sample_weight=w)
    pred = clf.predict(fit_space(X))
    export(clf, args.out)

    # the written file, evaluated by the library, must agree with scikit-learn
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    import paper_2506_20677_amd as ahs
    m = ahs.ahs_model_load(args.out)
    mism = 0
    regret = []
    for i in range(len(X)):
        f = ahs.FeatureVector(n=int(X[i, 0]), span=int(rows[i]["span"]), entropy_bits=float(X[i, 2]))
        c = ahs.ahs_model_predict(m, f) - ahs.COUNTING
        mism += int(c != pred[i])
        t = times[i]
        regret.append(t[c] / np.nanmin(t) if math.isfinite(t[c]) else float("inf"))
    acc = float(np.mean(pred == y))
    print(f"trained {len(clf.estimators_) * 3} trees on {len(X)} rows: accuracy {acc:.3f}, "
          f"mean time over best {np.mean([r for r in regret if math.isfinite(r)]):.4f}, "
          f"worst {max(regret):.3f}, library/scikit-learn disagreements {mism}")
    if mism:
        raise SystemExit("exported model does not reproduce the fitted classifier")


if __name__ == "__main__":
    main()
