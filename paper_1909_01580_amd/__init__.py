"""MI355X-native HGKS time stage (WENO-AO reconstruction, BGK face flux,
two-stage fourth-order update) behind a C-ABI library.

Importing the package loads nothing native; ``paper_1909_01580_amd.hgks``
binds the shared library and raises if it has not been built.
"""
