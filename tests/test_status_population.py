"""CPU check of the crafted status population used by the GPU status tests:
the oracle must take each of its Newton outcomes on it, else the GPU
comparison would not exercise them."""
from tests.test_gpu_status import test_population_exercises_every_newton_safeguard_in_the_oracle  # noqa: F401
