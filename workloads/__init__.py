"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package only *describes* inputs: grid sizes, boxes, symbolic
sum-of-products terms, initial-packet parameters and seeded random draws.
It performs none of the method's arithmetic (no DVR matrices, no potential
values, no propagation), so both sides evaluate every model quantity with
their own independent code.
"""
from .cards import card, CARD_NAMES  # noqa: F401
from .random_inputs import random_active_set, random_complex, random_dense_factor  # noqa: F401
