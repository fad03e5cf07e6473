"""MI355X-native BCFW solver for quadratic semi-relaxed optimal transport."""
