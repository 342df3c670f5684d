"""MI355X-native hot path of a pivoting-free primal-dual interior-point method.

Importing the package loads nothing native; the HIP library is loaded on first
use by :mod:`paper_2508_16094_amd.lib` and fails loudly when it is missing.
"""
