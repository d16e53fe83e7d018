"""MI355X-native manufactured-solution PIC/DSMC time step (HIP, gfx950).

Importing the package loads nothing; ``paper_2602_15130_amd.pic`` loads the
compiled HIP library and fails loudly if it is missing.
"""
