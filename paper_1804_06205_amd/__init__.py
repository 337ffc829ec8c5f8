"""MI355X-native DPD step library (arXiv 1804.06205, Groot-style DPD with
per-step cell binning and extra 1-3 / 1-5 Morse terms)."""
