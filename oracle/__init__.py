"""Serial FP64 CPU oracle of the WAKE quasi-static plasma response.

Test infrastructure only: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
