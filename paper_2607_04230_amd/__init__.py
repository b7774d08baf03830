"""MI355X-native deferred software rasterization of strand hair."""
