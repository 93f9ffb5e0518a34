"""MI355X-native plane-wave block-eigensolver step (HIP kernels behind a C ABI)."""
