"""MI355X-native Q-adic transform (FQT) library: DQT packing, exact FP64 MFMA
contraction and REDQ unpacking over GF(p^k), after J.-G. Dumas, "Q-adic
Transform Revisited".  The compute path is libfqt.so (HIP, gfx950); the
``fqt`` module is its binding."""
