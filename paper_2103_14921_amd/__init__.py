"""MI355X-native FD-Helmholtz ORAS-FGMRES solver (HIP library + thin binding).

``from paper_2103_14921_amd import helm`` loads the in-tree ``libhelm.so`` and
raises if it has not been built (``paper_2103_14921_amd.build.build()``).
"""
