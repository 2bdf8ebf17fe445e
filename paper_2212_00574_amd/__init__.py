"""MI355X-native colour-index kernelization for the k-clique problem.

The HIP library (libkz.so, C ABI in include/kz.h) does all the work; the
``binding`` module marshals PyTorch device tensors into it.  ``inputs`` holds
the seeded synthetic graph generators.
"""
