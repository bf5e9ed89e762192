"""Pins for the k-NN classification oracle (``oracle/classify.py``): the
hand-worked votes on the line (ties included), k = 1 giving the nearest
reference's label, invariance under a renaming of the classes, and a
brute-force vote over explicitly sorted distances (numpy argsort, not the C
oracle).  The last test plants mistakes (ties to the smallest class id, ties
to the farthest member) and checks that the pins catch them."""
from __future__ import annotations

import json
import os

import numpy as np

import synthdata
from oracle import classify as C

HERE = os.path.dirname(os.path.abspath(__file__))


def fixture_failures(classify_fn):
    with open(os.path.join(HERE, "golden", "classify_line.json")) as f:
        g = json.load(f)
    R = np.array(g["references"], dtype=np.float32)[:, None]
    lab = np.array(g["labels"])
    bad = 0
    for c in g["cases"]:
        Q = np.array([[c["query"]]], dtype=np.float32)
        bad += int(classify_fn(Q, R, lab, c["k"])[0]) != c["label"]
    return bad


def test_hand_worked_votes():
    assert fixture_failures(C.classify) == 0


def test_k1_is_nearest_label():
    Q = synthdata.uniform((50, 4), 11, 1)
    R = synthdata.uniform((400, 4), 11, 0)
    lab = np.random.default_rng(0).integers(0, 5, 400)
    d2 = ((Q[:, None, :].astype(np.float64) - R[None, :, :]) ** 2).sum(-1)
    nn = np.lexsort((np.broadcast_to(np.arange(400), d2.shape), d2), axis=1)[:, 0]
    assert np.array_equal(C.classify(Q, R, lab, 1), lab[nn])


def test_renaming_classes_renames_predictions():
    Q = synthdata.uniform((80, 3), 12, 1)
    R = synthdata.uniform((600, 3), 12, 0)
    lab = np.random.default_rng(1).integers(0, 6, 600)
    perm = np.random.default_rng(2).permutation(6)
    assert np.array_equal(perm[C.classify(Q, R, lab, 7)], C.classify(Q, R, perm[lab], 7))


def brute_force_failures(classify_fn):
    Q = synthdata.uniform((60, 2), 13, 1)
    R = synthdata.uniform((300, 2), 13, 0)
    lab = np.random.default_rng(3).integers(0, 4, 300)
    k = 6
    pred = classify_fn(Q, R, lab, k)
    bad = 0
    for i in range(Q.shape[0]):
        d2 = ((Q[i].astype(np.float64) - R.astype(np.float64)) ** 2).sum(-1)
        order = np.lexsort((np.arange(300), d2))[:k]
        counts = np.bincount(lab[order], minlength=4)
        tied = set(np.flatnonzero(counts == counts.max()))
        expect = next(int(lab[j]) for j in order if lab[j] in tied)
        bad += int(pred[i]) != expect
    return bad


def test_brute_force_vote():
    assert brute_force_failures(C.classify) == 0


def test_pins_catch_planted_mistakes():
    def smallest_id(Q, R, lab, k):  # ties to the smallest class id
        from oracle import knn

        _, idx = knn(Q, R, k, "l2")
        out = []
        for row in idx:
            c = np.bincount(lab[row])
            out.append(int(np.flatnonzero(c == c.max())[0]))
        return np.array(out)

    def farthest(Q, R, lab, k):  # ties to the farthest member of the tied classes
        from oracle import knn

        _, idx = knn(Q, R, k, "l2")
        return np.array([C.vote(list(lab[row])[::-1]) for row in idx])

    assert fixture_failures(smallest_id) + brute_force_failures(smallest_id) > 0
    assert fixture_failures(farthest) + brute_force_failures(farthest) > 0
