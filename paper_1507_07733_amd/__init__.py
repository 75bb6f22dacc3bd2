"""MI355X-native antenna-pattern unfolding (radio E-field reconstruction).

Importing the package is cheap: the HIP library is loaded on first use of
:mod:`paper_1507_07733_amd.api`.  :mod:`paper_1507_07733_amd.synth` holds the
seeded synthetic-input generators.
"""
__all__ = ["synth", "api"]
