"""MI355X-native finite-solid-angle GR radiation step (HIP kernels behind a C ABI)."""
