"""MI355X-native real-space FLOSIC self-interaction-correction path.

Importing the package loads nothing; the HIP library is loaded on first use
of :mod:`paper_2108_01186_amd.fsic`.
"""
