"""FP64 CPU oracle of AltGDmin-LR+S (arXiv 2311.03824), written from the paper.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
