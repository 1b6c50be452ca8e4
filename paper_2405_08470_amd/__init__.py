"""MI355X-native sparse MTTKRP with per-mode partitioning and dynamic remapping."""
