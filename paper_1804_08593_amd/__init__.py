"""MI355X-native multisplitting-preconditioned CG for domain-wall fermions."""
