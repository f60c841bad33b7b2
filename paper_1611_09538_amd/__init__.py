"""MI355X-native Spectral Ewald for singly periodic domains (SE1P)."""
