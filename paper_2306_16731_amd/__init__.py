"""MI355X-native Finite Volume patch update (Rusanov, compressible Euler, FP64)."""
