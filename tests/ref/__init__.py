"""Independent test references (textbook solutions), used only by tests."""
