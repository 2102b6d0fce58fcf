"""MI355X-native relativistic space-charge FMM (arXiv 2302.07567)."""
