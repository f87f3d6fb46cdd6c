"""MI355X-native exhaustive RKN seed scan for drift-chamber track finding."""
