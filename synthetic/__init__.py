"""Seeded synthetic lightcurves and templates.

This package only draws inputs (times, values, uncertainties, template
coefficients, frequency grids).  It holds none of the periodogram's
arithmetic, so both the CPU oracle and the GPU path may use it.
"""
from .lightcurves import *  # noqa: F401,F403
