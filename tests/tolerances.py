"""Tolerances shared by the GPU parity tests.

NEAR_TIE: a GPU decision may differ from the oracle's only where the
oracle's own cost at the GPU's choice is within the selection rule's tie
band of the cost it chose.  The GPU's FP64 window sums carry a relative
error below 6e-14 (the reseeded Gaussian recurrence bounds each weight's
error by 5.7e-14; the window's dropped tail is below 1e-16 of the sum), so
its band edge sits within 2 x 6e-14 of the oracle's: a differing choice costs
at most (1 + tau + 1.2e-13) times the oracle's, tau being the band (1e-12
unless the search sets another).
"""
TAU64 = 1e-12
EPS64 = 6e-14


def near_tie(tau=TAU64):
    return tau + 2 * EPS64
