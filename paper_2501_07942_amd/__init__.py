"""MI355X-native tensor-train grid-based filter (HIP library + thin binding)."""
