"""CPU oracle for the Monte Carlo sparse approximate inverse.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product library never does, and this
package never imports the product library. See ``mcmi_oracle.c`` for the
algorithm and ``ref.py`` for the Python wrapper and the numpy reference pieces.
"""
from .ref import *  # noqa: F401,F403
