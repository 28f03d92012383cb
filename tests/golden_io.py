"""Readers for the paper fixtures under tests/golden (1-based ids in files, 0-based returned)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def _set(tok):
    return set() if tok == "-" else {int(t) for t in tok.split(",")}


def fig1_graph():
    n, src, dst = None, [], []
    for r in _rows("fig1_graph.txt"):
        if r[0] == "n":
            n = int(r[1])
        else:
            src.append(int(r[0]) - 1)
            dst.append(int(r[1]) - 1)
    return n, np.array(src, np.uint32), np.array(dst, np.uint32)


def fig1_labels():
    """landmarks (0-based list), bucket table (uint8[n]) and per-vertex label sets."""
    n = fig1_graph()[0]
    landmarks, bucket, rows = None, np.zeros(n, np.uint8), {}
    for r in _rows("fig1_labels.txt"):
        if r[0] == "landmarks":
            landmarks = [int(t) - 1 for t in r[1:]]
        elif r[0] == "bucket":
            bucket[int(r[1]) - 1] = int(r[2])
        else:
            rows[int(r[0]) - 1] = tuple(_set(t) for t in r[1:5])
    return landmarks, bucket, rows


def fig3_insert():
    edge, rows = None, {}
    for r in _rows("fig3_insert.txt"):
        if r[0] == "insert":
            edge = (int(r[1]) - 1, int(r[2]) - 1)
        else:
            rows[int(r[0]) - 1] = (_set(r[1]), _set(r[2]))
    return edge, rows


def examples():
    return [(int(r[0]) - 1, int(r[1]) - 1, int(r[2]), r[3]) for r in _rows("examples.txt")]


def landmark_word(ids, landmarks):
    """Bit word of a set of 1-based landmark ids given the 0-based ordered landmark list."""
    w = 0
    for v in ids:
        w |= 1 << landmarks.index(v - 1)
    return w


def bucket_word(buckets):
    w = 0
    for b in buckets:
        w |= 1 << b
    return w
