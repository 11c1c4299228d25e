"""CPU tests of the benchmark's FP64x3 sampled check (bench.td_sampled_check):
entries taken from the full oracle pass, a planted 2^-60 relative error in
the second word does not."""
import numpy as np

import bench
from oracle.cascade3 import cascade3_gemm
from paper_2303_04353_amd.inputs import make_problem3, sample_entries


def test_td_sampled_check_accepts_the_oracle_and_rejects_a_planted_error():
    n, k = 24, 600
    P = make_problem3(n, n, k, cfg=9)
    O = cascade3_gemm(P["A"], P["B"], P["C"], kc=256)
    I, J = sample_entries(n, n, 16, seed=3)
    S = [O[w][I, J] for w in range(3)]
    r = bench.td_sampled_check(P, I, J, S)
    assert r["within_order_bound"] and r["entries"] == 16
    assert r["max_diff_from_oracle_over_absAabsB"] < 2.0 ** -140
    bad = [S[0], S[1] + S[0] * 2.0 ** -60, S[2]]
    assert not bench.td_sampled_check(P, I, J, bad)["within_order_bound"]
