"""MI355X-native block Krylov + operator action data path (HIP kernels behind a C ABI)."""
