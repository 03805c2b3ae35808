"""CPU oracle of the occlusion detector -- TEST INFRASTRUCTURE.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library neither links nor calls it,
and it shares no code with the GPU path.
"""
