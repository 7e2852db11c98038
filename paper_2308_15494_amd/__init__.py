"""MI355X-native unconstrained partition refinement (one synchronous round).

Importing the package loads nothing native; the HIP library is loaded on
first use by :mod:`paper_2308_15494_amd.upr`.
"""
