"""Pin of the storage accounting against the byte counts the paper prints
(tests/golden/paper_storage.json)."""
import json
import os

from oracle import storage

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_storage.json")))


def test_rank50_factor_counts():
    g = GOLD["lenna_rank50"]
    v = storage.factor_values(g["m"], g["n"], g["k"])
    assert v == g["values"]
    assert storage.values_bytes(v, "f16") == g["bytes_half"]
    assert storage.values_bytes(v, "f64") == g["bytes_double"]


def test_dense_sizes_of_the_sparse_test_matrices():
    tib = 2.0 ** 40
    h = storage.dense_bytes(GOLD["hamrle3_dense"]["n"], GOLD["hamrle3_dense"]["n"], "f64") / tib
    c = storage.dense_bytes(GOLD["circuit5m_dense"]["n"], GOLD["circuit5m_dense"]["n"], "f64") / tib
    assert h > GOLD["hamrle3_dense"]["more_than_TB"]
    assert abs(c - GOLD["circuit5m_dense"]["roughly_TB"]) / GOLD["circuit5m_dense"]["roughly_TB"] < 0.01
