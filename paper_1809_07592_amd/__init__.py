"""MI355X-native Toeplitz-hash privacy amplification (binding filled in below)."""
