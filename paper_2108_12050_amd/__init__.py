"""MI355X-native MHFD scale-space LoG focus detector (placeholder)."""
