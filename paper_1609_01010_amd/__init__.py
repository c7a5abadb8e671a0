"""MI355X-native modular polynomial multiplication (NTT / TFT convolution)."""
