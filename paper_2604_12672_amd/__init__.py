"""MI355X-native explicit finite-volume MHD step (PHLEGETHON hot path).

Importing the package loads nothing; ``paper_2604_12672_amd.mhd`` binds the
HIP library.
"""
