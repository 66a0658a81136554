"""The shipped selector (gradient-boosted trees of Sec. III-H trained on
MI355X measurements, models/mi355x_selector.gbt): the library and the
oracle parse it and reach the same decision on every labelled workload,
both through the predictor alone and through the full decision engine with
the model enabled; and its decisions stay close to the measured best."""
import csv
import math
import os

import pytest

import oracle as O

ahs = pytest.importorskip("paper_2506_20677_amd")

LABELS = os.path.join(os.path.dirname(ahs.SELECTOR_MODEL), "mi355x_labels.csv")
NAMES = ("counting", "radix", "quick")


def rows():
    return list(csv.DictReader(open(LABELS)))


def test_library_and_oracle_agree_on_every_labelled_workload():
    lm = ahs.default_model()
    om = O.Model(ahs.SELECTOR_MODEL)
    lcfg = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    ocfg = O.config(0, use_model=1)
    for r in rows():
        n, span, H = int(r["n"]), int(r["span"]), float(r["entropy_bits"])
        lf = ahs.FeatureVector(n=n, span=span, entropy_bits=H, nbins=int(r["nbins"]))
        of = O.Features(n=n, span=span, entropy_bits=H, nbins=int(r["nbins"]))
        assert ahs.ahs_model_predict(lm, lf) == om.predict(of), r
        st, oc = O.select(of, ocfg, om)
        assert st == O.OK
        assert ahs.ahs_select(lf, lcfg, lm) == oc, r


def test_model_decisions_cost_little_over_the_measured_best():
    om = O.Model(ahs.SELECTOR_MODEL)
    regret = []
    for r in rows():
        f = O.Features(n=int(r["n"]), span=int(r["span"]), entropy_bits=float(r["entropy_bits"]))
        c = NAMES[om.predict(f) - O.COUNTING]
        t = {k: float(r[f"t_{k}"]) for k in NAMES}
        assert math.isfinite(t[c]), r  # never counting where counting is refused
        regret.append(t[c] / min(t.values()))
    assert sum(regret) / len(regret) < 1.02
    assert max(regret) < 2.0
