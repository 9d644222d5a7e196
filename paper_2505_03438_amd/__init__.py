"""MI355X-native short-range Lennard-Jones MD hot path (HIP for gfx950).

Importing the package loads nothing; ``paper_2505_03438_amd.mdlj`` loads the
HIP library on first use and raises if it is missing.
"""
