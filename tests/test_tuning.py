"""Parameter choice for a required accuracy (host logic; no device needed)."""
from paper_1811_12498_amd.tuning import Candidate, select


def test_select_fastest_accurate_enough():
    t = [Candidate(4, 0.7, 500, 3.0, 2e-4), Candidate(6, 0.6, 500, 4.0, 4e-5),
         Candidate(8, 0.5, 1000, 5.0, 5e-6), Candidate(6, 0.5, 2000, 3.5, 9e-6),
         Candidate(10, 0.4, 1000, 9.0, 1e-7)]
    assert select(t, 1e-3) == t[0]
    assert select(t, 5e-5) == t[3]
    assert select(t, 9e-6) == t[3]
    assert select(t, 8e-6) == t[2]
    assert select(t, 1e-7) == t[4]
    assert select(t, 1e-8) is None
    assert select([], 1.0) is None


def test_select_ties_prefer_smaller_error_then_order():
    t = [Candidate(8, 0.5, 1000, 2.0, 3e-6), Candidate(6, 0.5, 1000, 2.0, 1e-6),
         Candidate(4, 0.5, 1000, 2.0, 1e-6)]
    assert select(t, 1e-5) == t[2]
