"""CPU oracle of the MGFWA hot path -- TEST INFRASTRUCTURE ONLY.

Imported only by tests/, the smoke check and the benchmark's CPU-baseline leg;
the product library never loads it.
"""
from .oracle import Oracle, Problem, explosion_row, init_row, make_config, philox, u01, word  # noqa: F401
