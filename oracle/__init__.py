"""FP64 CPU oracle of pruned wavepacket propagation.

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.
"""
