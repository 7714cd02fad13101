"""MI355X-native inverse ray-shooting of microlensing magnification maps."""
