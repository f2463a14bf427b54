"""MI355X-native strong-field QED step (arXiv:1412.6426) behind a C-ABI library."""
