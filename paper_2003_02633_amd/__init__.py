"""MI355X-native inline 3-vector compression (arXiv 2003.02633)."""
