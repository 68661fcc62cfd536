"""CPU oracle of the muon trigger.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  ``literal`` is a pure-Python rendering of the rule for
tiny slices; ``cpu`` drives the C oracle (strict all-pairs and blocked forms).
"""
