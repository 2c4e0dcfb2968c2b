"""The CPU oracle: a plain, slow implementation of what the path computes,
written from the paper. TEST INFRASTRUCTURE ONLY: tests/, the smoke entry
point and the benchmark's CPU-baseline leg use it; the product path never
imports it."""
