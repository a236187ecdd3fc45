"""MI355X-native accurate eigensolver for real symmetric arrowhead matrices."""
