"""MI355X-native pseudo-spectral compressible-MHD hot path (HIP kernels behind a C-ABI)."""
