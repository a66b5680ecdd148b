"""FP64 CPU oracle of the agent-based optimal-control solver.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports or calls it.
"""
