"""MI355X-native subspace culling for BVH ray traversal (Yoshimura & Harada 2023).

Importing the package is cheap: the HIP library is loaded on first use of
:mod:`paper_2305_08343_amd.binding`.
"""
