"""MI355X-native batched rMD / SCPS stepping (Self-Consistent Path Sampling).

Importing the package does not load the HIP library; ``paper_1705_02180_amd.scps``
does, and fails loudly when the library has not been built.
"""
