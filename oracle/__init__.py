"""CPU oracle of the census template-matching path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package. The library path never imports it.
"""
