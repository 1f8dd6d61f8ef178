"""Each deliberate mistake planted in the oracle is caught by the named pins.

Mutations (planted inside the oracle only, switched by a test hook):
1 Gaussian derivative sign flipped; 2 stratified zeros not rejected;
3 semi-stratified "zero" weight zeta/q instead of omega/q; 4 semi-stratified
nonzero correction -g(0,m) dropped; 5 the wrong factor left out of the
Khatri-Rao row; 6 Adam epsilon moved outside the square root; 7 weighted
semi-stratified correction uses the entry's own weight instead of w_zero;
8 the loss estimate weights a stratified zero by omega/q instead of zeta/q
(the gradient keeps the right weight); 9 GCP-Adam's undo leaves the step
count where the undone epoch ended.
"""
import pytest

import oracle
import pins

EXPECTED = {
    1: {"gaussian_closed_form", "fd_gaussian"},
    2: {"sample_streams", "stratified_zeros_are_zeros", "unbiased_stratified_bernoulli"},
    3: {"unbiased_semi_bernoulli", "semi_zero_half_poisson"},
    4: {"unbiased_semi_bernoulli", "fd_poisson_semi"},
    5: {"enumeration_equals_unfolding", "gaussian_closed_form", "poisson_closed_form"},
    6: {"adam_closed_forms"},
    7: {"weighted_unbiased_semi"},
    8: {"loss_estimate_stratified", "loss_estimate_weighted_stratified"},
    9: {"adam_fit_rewind"},
}


@pytest.mark.parametrize("mutation", sorted(EXPECTED))
def test_planted_mistake_is_caught(mutation):
    oracle.set_mutation(mutation)
    try:
        failed = {name for name in EXPECTED[mutation] if not pins.ALL_PINS[name]()[0]}
    finally:
        oracle.set_mutation(0)
    assert failed == EXPECTED[mutation], f"mutation {mutation}: only {failed} caught it"
